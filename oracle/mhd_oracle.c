/*
 * FP64 CPU oracle for the single-step simplified lattice Boltzmann scheme of quasi-static MHD
 * pipe flow (Tavares, Magacho, Moriconi, Loureiro, arXiv:2211.09370).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path links, loads or calls this file: it is
 * built into its own shared object and used by the tests, by the smoke check and by the timed
 * CPU baseline of the benchmark. It shares no source, header, table or helper with the HIP
 * library.
 *
 * Everything here is written out the slow, literal way: every equilibrium is formed in full at
 * the cell it belongs to and gathered from the neighbour named by the update formula; no moment
 * shortcuts, no fusion. Arithmetic is IEEE double; build with -ffp-contract=off.
 *
 * Lattice: D3Q19 (rest 1/3, six faces 1/18, twelve edges 1/36, c_s^2 = 1/3) or the paper's D3Q27
 * (rest 8/27, faces 2/27, edges 1/54, corners 1/216) for every part of the step, box nx*ny*nz
 * periodic on every face, fields component-major with x fastest.
 *
 * Step n -> n+1 (Sec. 5.7: the magnetic iteration runs before each velocity update):
 *   1. N_mag times: b* = sum_i g_i^eq(x - e_i)      (tau_m = 1 macroscopic update, Sec. 5.7)
 *                   b  = b* + D^T S_m (b_wall - D b*) (explicit IB for B, Sec. 5.4 / 5.6)
 *   2. F = G(t) x + (curl b) x (B_ext + b)           (Lorentz force, Sec. 5.1)
 *   3. rho', u* from the single-step update with the GZS forcing and its lattice discrete-effect
 *      term (Sec. 3.3 and Sec. 5.1), optionally with the time-step rescaling gamma of Sec. 7;
 *      for tau >= 1 from the macroscopic tau = 1 update with particle speed 6 nu (Sec. 5.7)
 *   4. u = u* + D^T S (u_wall - D u*)                (explicit IB for u, Sec. 5.3 / 5.5)
 *   5. optional flow-rate control of G, t += 1.
 *
 * Readings where the paper is silent or ambiguous (each listed in the design notes):
 *   - the magnetic unknown is the induced field b; diffusion acts on b and the advection flux
 *     uses B = B_ext + b (identical to the paper's total-B iteration when lap(B_ext) = 0);
 *   - the Lorentz current is J = curl b (identical for curl-free B_ext);
 *   - the improved momentum update is read in momentum form: rho' u* = gather - (tau/2) sum ...
 *     + F, as in the plain forcing form of Sec. 3.5;
 *   - with the rescaling gamma (Sec. 7) the explicit force term is F dt with the rescaled step
 *     dt = 1/gamma, so that a steady state does not depend on gamma;
 *   - the macroscopic branch (tau >= 1) takes the GZS forcing at tau = 1 with the usual half-force
 *     term in the momentum, (dt/2) F(x), evaluated with the force of the current step;
 *   - the wall correction for B runs after every magnetic sweep, the one for u once per step;
 *   - sums over i run over all Q directions, rest included;
 *   - the Lagrange stencil of a marker is its nearest node and that node +-1 in each direction,
 *     ties at |r| = 1/2 broken by n0 = floor(X + 1/2); taps with weight exactly 0 are skipped.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------ */
/* Parameters (mirrored field by field by a ctypes Structure in oracle/__init__.py)           */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int nx, ny, nz;
    double nu, eta;
    int n_mag;
    double lambda_u, lambda_b;
    double G0, G1, period;
    int bext_kind; /* 0 none, 1 uniform along y, 2 tanh fringe along y, 3 six magnets */
    double B0, fringe_x0, fringe_w;
    double yc, zc, radius;
    int flow_control;
    double u_target, k_c;
    int ib_u, ib_b; /* 1 = apply the wall correction for u / for b */
    double alpha;   /* accelerated magnetic iteration (Sec. 5.8); <= 0 means 1 (plain sweep) */
    double magnet_L, magnet_D; /* six magnets: strip half-width (<= 0: radius / 6) and distance
                                  of the strip centres from the axis (<= 0: see magnet_geometry) */
    int lattice;    /* 27: D3Q27 (the paper's set, Table I); otherwise D3Q19 */
    double gamma;   /* time-step rescaling of Sec. 7 (dt -> dt / gamma); <= 0 means 1 */
    double omega_radius; /* budget region Omega = {r < omega_radius}; <= 0 means radius - 2 */
} orc_params;

/* D3Q19 velocity set and weights (textbook values). */
static const int E19[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double W19[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* D3Q27 (the paper's set): the tensor product of the 1D weights (2/3, 1/6, 1/6) -> rest 8/27,
 * six faces 2/27, twelve edges 1/54, eight corners 1/216. */
static const int E27[27][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
static const double W27[27] = {
    8.0 / 27.0,
    2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
    1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
    1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
    1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0};
static const double CS2 = 1.0 / 3.0;

/* The velocity set in use: Q velocities E[i], weights W[i] (rest first). */
typedef struct {
    int Q;
    const int (*E)[3];
    const double *W;
} lattice_t;
static inline lattice_t lattice_of(const orc_params *p) {
    lattice_t l;
    if (p->lattice == 27) {
        l.Q = 27;
        l.E = E27;
        l.W = W27;
    } else {
        l.Q = 19;
        l.E = E19;
        l.W = W19;
    }
    return l;
}

static inline int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

static inline int64_t cell(const orc_params *p, int x, int y, int z) {
    return (int64_t)wrap(x, p->nx) + (int64_t)p->nx * ((int64_t)wrap(y, p->ny) + (int64_t)p->ny * wrap(z, p->nz));
}

static inline int64_t ncells(const orc_params *p) { return (int64_t)p->nx * p->ny * p->nz; }

/* Field of one magnet in its own frame (Sec. 6, Biot-Savart form): a strip of half-width L on
 * z' = 0, |y'| < L; B_y' = 2 [atan((y' - L)/z') - atan((y' + L)/z')],
 * B_z' = log(((y' + L)^2 + z'^2) / ((y' - L)^2 + z'^2)). */
static void magnet_local(double yl, double zl, double L, double out[2]) {
    out[0] = 2.0 * (atan((yl - L) / zl) - atan((yl + L) / zl));
    out[1] = log(((yl + L) * (yl + L) + zl * zl) / ((yl - L) * (yl - L) + zl * zl));
}

/* Six magnets with alternating poles on a hexagon around the pipe axis (yc, zc): magnet m sits at
 * angle 60 m degrees, distance D, its strip tangential and its z' axis pointing radially
 * outwards, polarity (-1)^m. L defaults to R / 6 (Sec. 6); D defaults to the distance of the
 * farthest cell of the box from the axis plus L + 1, so no strip reaches into the box. */
static void magnet_geometry(const orc_params *p, double *L, double *D) {
    *L = p->magnet_L > 0.0 ? p->magnet_L : p->radius / 6.0;
    if (p->magnet_D > 0.0) {
        *D = p->magnet_D;
    } else {
        double dy = fmax(p->yc, (double)(p->ny - 1) - p->yc), dz = fmax(p->zc, (double)(p->nz - 1) - p->zc);
        *D = sqrt(dy * dy + dz * dz) + *L + 1.0;
    }
}

static void six_magnets_raw(const orc_params *p, double y, double z, double B[2]) {
    double L, D;
    magnet_geometry(p, &L, &D);
    B[0] = B[1] = 0.0;
    for (int m = 0; m < 6; ++m) {
        double th = m * (3.14159265358979323846 / 3.0);
        double n[2] = {cos(th), sin(th)}, t[2] = {-sin(th), cos(th)};
        double ry = y - (p->yc + D * n[0]), rz = z - (p->zc + D * n[1]);
        double yl = ry * t[0] + rz * t[1], zl = ry * n[0] + rz * n[1];
        double f[2];
        magnet_local(yl, zl, L, f);
        double sgn = (m % 2 == 0) ? 1.0 : -1.0;
        B[0] += sgn * (f[0] * t[0] + f[1] * n[0]);
        B[1] += sgn * (f[0] * t[1] + f[1] * n[1]);
    }
}

/* Imposed field B_ext at a point (x, y, z) of the box (any real coordinates). Six magnets:
 * scaled so that |B| = B0 at the wall point (yc + R, zc) facing magnet 0. */
void orc_bext_at(const orc_params *p, double x, double y, double z, double B[3]) {
    B[0] = B[1] = B[2] = 0.0;
    if (p->bext_kind == 1) {
        B[1] = p->B0;
    } else if (p->bext_kind == 2) {
        B[1] = p->B0 * 0.5 * (1.0 + tanh((x - p->fringe_x0) / p->fringe_w));
    } else if (p->bext_kind == 3) {
        double f[2], r[2];
        six_magnets_raw(p, y, z, f);
        six_magnets_raw(p, p->yc + p->radius, p->zc, r);
        double s = p->B0 / sqrt(r[0] * r[0] + r[1] * r[1]);
        B[1] = s * f[0];
        B[2] = s * f[1];
    }
}

/* Imposed field at cell (x, y, z). */
void orc_bext(const orc_params *p, int x, int y, int z, double B[3]) {
    orc_bext_at(p, (double)x, (double)y, (double)z, B);
}

/* ------------------------------------------------------------------------------------------ */
/* Equilibria                                                                                 */
/* ------------------------------------------------------------------------------------------ */

/* Fluid equilibrium f_i^eq(rho, u) with c_s^2 = 1/3 (Sec. 3.1 / Sec. 3.5). With the time-step
 * rescaling of Sec. 7 (dt -> dt / gamma, c_i -> gamma c_i) the quadratic part is divided by
 * gamma; gamma = 1 is the plain equilibrium. */
static inline double feq(const lattice_t *L, int i, double rho, const double u[3], double gamma) {
    const int *e = L->E[i];
    double cu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double quad = (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
    return L->W[i] * rho * (1.0 + cu / CS2 + quad / gamma);
}

/* GZS forcing population F_i (Sec. 5.1), in the rescaled form of Sec. 7:
 * (1 - 1/(2 tau)) w_i [(c_i - u/gamma) / (gamma c_s^2) + (c_i . u) c_i / (gamma^2 c_s^4)] . F
 * (gamma = 1: the plain GZS population). */
static inline double fgzs(const lattice_t *L, int i, double tau, double gamma, const double u[3],
                          const double F[3]) {
    const int *e = L->E[i];
    double cu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
    double s = 0.0;
    for (int a = 0; a < 3; ++a) {
        double v = (e[a] - u[a] / gamma) / (gamma * CS2) + cu * e[a] / (gamma * gamma * CS2 * CS2);
        s += v * F[a];
    }
    return (1.0 - 1.0 / (2.0 * tau)) * L->W[i] * s;
}

/* Equilibrium with particle speed c (c_i = c e_i, c_s^2 = c^2 / 3), the macroscopic branch of
 * Sec. 5.7 for tau >= 1. */
static inline double feq_c(const lattice_t *L, int i, double c, double rho, const double u[3]) {
    double ci[3], cs2 = c * c / 3.0;
    for (int a = 0; a < 3; ++a) ci[a] = c * L->E[i][a];
    double cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2];
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return L->W[i] * rho * (1.0 + cu / cs2 + (cu * cu) / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
}

/* GZS population with particle speed c and tau = 1: (1/2) w_i [(c_i - u)/c_s^2 + (c_i . u) c_i /
 * c_s^4] . F. */
static inline double fgzs_c(const lattice_t *L, int i, double c, const double u[3], const double F[3]) {
    double ci[3], cs2 = c * c / 3.0;
    for (int a = 0; a < 3; ++a) ci[a] = c * L->E[i][a];
    double cu = ci[0] * u[0] + ci[1] * u[1] + ci[2] * u[2];
    double s = 0.0;
    for (int a = 0; a < 3; ++a) s += ((ci[a] - u[a]) / cs2 + cu * ci[a] / (cs2 * cs2)) * F[a];
    return 0.5 * L->W[i] * s;
}

/* Magnetic equilibrium of the tau_m = 1 iteration with particle speed c = 6 eta (Sec. 5.7):
 * g_{i,a} = w_i [ b_a + sum_c (c_ic / cs_m^2) (u_c B_a - u_a B_c) ], c_i = c e_i, cs_m^2 = c^2/3.
 * `b` is the induced field, B = B_ext + b enters the flux. */
static inline void geq(const lattice_t *L, int i, double c, const double u[3], const double b[3],
                       const double B[3], double g[3]) {
    double csm2 = c * c / 3.0;
    for (int a = 0; a < 3; ++a) {
        double s = b[a];
        for (int cc = 0; cc < 3; ++cc) {
            double cic = c * L->E[i][cc];
            s += (cic / csm2) * (u[cc] * B[a] - u[a] * B[cc]);
        }
        g[a] = L->W[i] * s;
    }
}

static inline void load3(const double *f, int64_t N, int64_t k, double v[3]) {
    v[0] = f[k];
    v[1] = f[N + k];
    v[2] = f[2 * N + k];
}

/* ------------------------------------------------------------------------------------------ */
/* Magnetic sweep: b*(x) = sum_i g_i^eq(x - e_i)  (Sec. 5.7, tau_m = 1, c = 6 eta)            */
/* ------------------------------------------------------------------------------------------ */
void orc_mag_sweep(const orc_params *p, const double *u, const double *b, double *bout) {
    const int64_t N = ncells(p);
    const double c = 6.0 * p->eta;
    /* Sec. 5.8, eq. "magnetic field quasi-static acelerated": the rest population becomes
     * (w_0 - 1 + alpha) b and the gathered sum is divided by alpha (alpha = 1: Sec. 5.7). */
    const double alpha = p->alpha > 0.0 ? p->alpha : 1.0;
    const lattice_t L = lattice_of(p);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                double acc[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < L.Q; ++i) {
                    int sx = x - L.E[i][0], sy = y - L.E[i][1], sz = z - L.E[i][2];
                    int64_t k = cell(p, sx, sy, sz);
                    double us[3], bs[3], Bs[3], Be[3], g[3];
                    load3(u, N, k, us);
                    load3(b, N, k, bs);
                    orc_bext(p, wrap(sx, p->nx), wrap(sy, p->ny), wrap(sz, p->nz), Be);
                    for (int a = 0; a < 3; ++a) Bs[a] = Be[a] + bs[a];
                    geq(&L, i, c, us, bs, Bs, g);
                    if (i == 0)
                        for (int a = 0; a < 3; ++a) g[a] += (alpha - 1.0) * bs[a];
                    for (int a = 0; a < 3; ++a) acc[a] += g[a];
                }
                int64_t k0 = cell(p, x, y, z);
                for (int a = 0; a < 3; ++a) bout[a * N + k0] = acc[a] / alpha;
            }
}

/* ------------------------------------------------------------------------------------------ */
/* Immersed boundary (Sec. 5.2 - 5.6)                                                         */
/* ------------------------------------------------------------------------------------------ */

/* One-dimensional three-point Lagrange kernel D_x(r) of Sec. 5.2 evaluated on the three nodes
 * nearest to X: n0 = floor(X + 1/2) and n0 +- 1. Returns n0 - 1 and the weights of
 * nodes n0 - 1, n0, n0 + 1 (r = node - X). */
int orc_lagrange3(double X, double w[3]) {
    int n0 = (int)floor(X + 0.5);
    double r;
    r = (double)(n0 - 1) - X; /* in [-3/2, -1/2] */
    w[0] = 0.5 * (r + 1.0) * (r + 2.0);
    r = (double)n0 - X; /* in [-1/2, 1/2] */
    w[1] = 1.0 - r * r;
    r = (double)(n0 + 1) - X; /* in [1/2, 3/2] */
    w[2] = 0.5 * (r - 1.0) * (r - 2.0);
    return n0 - 1;
}

typedef struct {
    int ntap;
    int64_t idx[27];
    double w[27];
} orc_marker;

/* Nonzero taps of D(x_k - X_j) = D_x D_y D_z for one marker (periodic wrap). */
static void marker_taps(const orc_params *p, const double Xj[3], orc_marker *m) {
    double wx[3], wy[3], wz[3];
    int bx = orc_lagrange3(Xj[0], wx);
    int by = orc_lagrange3(Xj[1], wy);
    int bz = orc_lagrange3(Xj[2], wz);
    m->ntap = 0;
    for (int c = 0; c < 3; ++c)
        for (int bb = 0; bb < 3; ++bb)
            for (int a = 0; a < 3; ++a) {
                double w = wx[a] * wy[bb] * wz[c];
                if (w == 0.0) continue;
                m->idx[m->ntap] = cell(p, bx + a, by + bb, bz + c);
                m->w[m->ntap] = w;
                m->ntap++;
            }
}

/* Expose the taps of a marker (for the tests). Returns the number of taps. */
int orc_marker_taps(const orc_params *p, const double Xj[3], int64_t *idx, double *w) {
    orc_marker m;
    marker_taps(p, Xj, &m);
    for (int t = 0; t < m.ntap; ++t) {
        idx[t] = m.idx[t];
        w[t] = m.w[t];
    }
    return m.ntap;
}

/* Row sums d_j = sum_i A_ji of A = D D^T (Sec. 5.3). Since A_ji = sum_k D_jk D_ik, the row sum is
 * sum_k D_jk (sum_i D_ik): the inner sum is accumulated on the grid first. */
void orc_ib_rowsums(const orc_params *p, int64_t M, const double *X, double *d) {
    const int64_t N = ncells(p);
    double *S = (double *)calloc((size_t)N, sizeof(double));
    orc_marker m;
    for (int64_t j = 0; j < M; ++j) {
        double Xj[3] = {X[j], X[M + j], X[2 * M + j]};
        marker_taps(p, Xj, &m);
        for (int t = 0; t < m.ntap; ++t) S[m.idx[t]] += m.w[t];
    }
    for (int64_t j = 0; j < M; ++j) {
        double Xj[3] = {X[j], X[M + j], X[2 * M + j]};
        marker_taps(p, Xj, &m);
        double s = 0.0;
        for (int t = 0; t < m.ntap; ++t) s += m.w[t] * S[m.idx[t]];
        d[j] = s;
    }
    free(S);
}

/* Diagonal scaling of the explicit correction with the viscosity / resistivity ratio lambda
 * (Sec. 5.5 and 5.6): lambda / (d_j (1 + d_j (lambda - 1))). lambda = 1 gives 1/d_j (Sec. 5.3). */
static inline double ib_scale(double lambda, double dj) {
    return lambda / (dj * (1.0 + dj * (lambda - 1.0)));
}

/* phi = phi* + D^T diag(s) (phi_wall - D phi*), all three components, in place.
 * wall may be NULL (wall value 0). d holds the row sums of D D^T. */
void orc_ib_correct(const orc_params *p, int64_t M, const double *X, const double *d,
                    double lambda, const double *wall, double *phi) {
    const int64_t N = ncells(p);
    orc_marker *mk = (orc_marker *)malloc((size_t)M * sizeof(orc_marker));
    double *delta = (double *)malloc((size_t)(3 * M) * sizeof(double));
    /* interpolation from the predicted field and the Lagrangian correction */
    for (int64_t j = 0; j < M; ++j) {
        double Xj[3] = {X[j], X[M + j], X[2 * M + j]};
        marker_taps(p, Xj, &mk[j]);
        double sj = ib_scale(lambda, d[j]);
        for (int a = 0; a < 3; ++a) {
            double I = 0.0;
            for (int t = 0; t < mk[j].ntap; ++t) I += mk[j].w[t] * phi[a * N + mk[j].idx[t]];
            double target = wall ? wall[a * M + j] : 0.0;
            delta[a * M + j] = sj * (target - I);
        }
    }
    /* spreading to the Eulerian nodes, after every interpolation has been taken */
    for (int64_t j = 0; j < M; ++j)
        for (int a = 0; a < 3; ++a)
            for (int t = 0; t < mk[j].ntap; ++t)
                phi[a * N + mk[j].idx[t]] += mk[j].w[t] * delta[a * M + j];
    free(delta);
    free(mk);
}

/* ------------------------------------------------------------------------------------------ */
/* Lorentz + body force: F = G x + (curl_h b) x (B_ext + b), isotropic differences (Sec. 5.1)  */
/* ------------------------------------------------------------------------------------------ */

/* d_a phi(x) = (1/c_s^2) sum_i w_i e_ia phi(x + e_i) */
static inline void grad_iso(const orc_params *p, const double *f, int x, int y, int z, double g[3]) {
    const lattice_t L = lattice_of(p);
    g[0] = g[1] = g[2] = 0.0;
    for (int i = 1; i < L.Q; ++i) {
        double v = f[cell(p, x + L.E[i][0], y + L.E[i][1], z + L.E[i][2])];
        for (int a = 0; a < 3; ++a) g[a] += L.W[i] * L.E[i][a] * v;
    }
    for (int a = 0; a < 3; ++a) g[a] /= CS2;
}

/* lap phi(x) = (2/c_s^2) sum_i w_i (phi(x + e_i) - phi(x)) */
static inline double lap_iso(const orc_params *p, const double *f, int x, int y, int z) {
    const lattice_t L = lattice_of(p);
    double c0 = f[cell(p, x, y, z)], s = 0.0;
    for (int i = 1; i < L.Q; ++i) s += L.W[i] * (f[cell(p, x + L.E[i][0], y + L.E[i][1], z + L.E[i][2])] - c0);
    return 2.0 * s / CS2;
}

static inline void curl_iso(const orc_params *p, const double *b, int x, int y, int z, double J[3]) {
    const int64_t N = ncells(p);
    double gx[3], gy[3], gz[3];
    grad_iso(p, b, x, y, z, gx);
    grad_iso(p, b + N, x, y, z, gy);
    grad_iso(p, b + 2 * N, x, y, z, gz);
    J[0] = gz[1] - gy[2];
    J[1] = gx[2] - gz[0];
    J[2] = gy[0] - gx[1];
}

void orc_lorentz(const orc_params *p, const double *b, double G, double *F) {
    const int64_t N = ncells(p);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k = cell(p, x, y, z);
                double J[3], B[3], bb[3];
                curl_iso(p, b, x, y, z, J);
                orc_bext(p, x, y, z, B);
                load3(b, N, k, bb);
                for (int a = 0; a < 3; ++a) B[a] += bb[a];
                F[k] = G + (J[1] * B[2] - J[2] * B[1]);
                F[N + k] = J[2] * B[0] - J[0] * B[2];
                F[2 * N + k] = J[0] * B[1] - J[1] * B[0];
            }
}

/* ------------------------------------------------------------------------------------------ */
/* Fluid update                                                                               */
/* ------------------------------------------------------------------------------------------ */
static double gamma_of(const orc_params *p) { return p->gamma > 0.0 ? p->gamma : 1.0; }

/* Relaxation time of the fluid: nu = c_s^2 (tau - 1/2) dt with the rescaled step dt / gamma
 * (Sec. 7), i.e. tau = 3 nu / gamma + 1/2. */
double orc_fluid_tau(const orc_params *p) { return p->nu / (CS2 * gamma_of(p)) + 0.5; }

/* Single-step predictor with GZS forcing and discrete-effect term (Sec. 3.3, 5.1), tau < 1:
 *   rho'    = sum_i [3/2 f_i(x - e_i) - f_i(x) + 1/2 f_i(x + e_i)]
 *   rho' u' = sum_i e_i {f_i(x - e_i) + (tau - 1) [f_i(x + e_i) - 2 f_i(x) + f_i(x - e_i)]}
 *             - (tau/2) sum_i e_i [F_i(x + e_i) - F_i(x - e_i)] + F(x) dt
 * with the rescaled f^eq, F_i and tau of Sec. 7 and dt = 1/gamma (1 without rescaling). */
static void fluid_single_step(const orc_params *p, const double *rho, const double *u, const double *F,
                              double *rho_out, double *u_out) {
    const int64_t N = ncells(p);
    const double gamma = gamma_of(p);
    const double tau = orc_fluid_tau(p);
    const lattice_t L = lattice_of(p);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k0 = cell(p, x, y, z);
                double u0[3], F0[3];
                load3(u, N, k0, u0);
                load3(F, N, k0, F0);
                double rsum = 0.0, m[3] = {0.0, 0.0, 0.0}, fsum[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < L.Q; ++i) {
                    int64_t km = cell(p, x - L.E[i][0], y - L.E[i][1], z - L.E[i][2]);
                    int64_t kp = cell(p, x + L.E[i][0], y + L.E[i][1], z + L.E[i][2]);
                    double um[3], up[3], Fm[3], Fp[3];
                    load3(u, N, km, um);
                    load3(u, N, kp, up);
                    load3(F, N, km, Fm);
                    load3(F, N, kp, Fp);
                    double f_m = feq(&L, i, rho[km], um, gamma); /* f_i^eq(x - e_i) */
                    double f_0 = feq(&L, i, rho[k0], u0, gamma); /* f_i^eq(x) */
                    double f_p = feq(&L, i, rho[kp], up, gamma); /* f_i^eq(x + e_i) */
                    rsum += 1.5 * f_m - f_0 + 0.5 * f_p;
                    double Fi_p = fgzs(&L, i, tau, gamma, up, Fp);
                    double Fi_m = fgzs(&L, i, tau, gamma, um, Fm);
                    for (int a = 0; a < 3; ++a) {
                        m[a] += L.E[i][a] * (f_m + (tau - 1.0) * (f_p - 2.0 * f_0 + f_m));
                        fsum[a] += L.E[i][a] * (Fi_p - Fi_m);
                    }
                }
                rho_out[k0] = rsum;
                for (int a = 0; a < 3; ++a) {
                    double mom = m[a] - 0.5 * tau * fsum[a] + F0[a] / gamma;
                    u_out[a * N + k0] = mom / rsum;
                }
            }
}

/* Macroscopic update for tau >= 1 (Sec. 5.7): the BGK update with tau = 1 and the GZS forcing
 * population, particle speed c = 6 nu (c_i = c e_i, c_s^2 = c^2/3, dt = 1/c, dx = 1):
 *   f_i(x, t + dt) = f_i^eq(x - c_i dt, t) + dt F_i(x - c_i dt, t)
 *   rho' = sum_i f_i(x, t + dt),  rho' u' = sum_i c_i f_i(x, t + dt) + (dt/2) F(x, t).
 * One call advances the time by dt = 1/(6 nu). */
static void fluid_macroscopic(const orc_params *p, const double *rho, const double *u, const double *F,
                              double *rho_out, double *u_out) {
    const int64_t N = ncells(p);
    const double c = 6.0 * p->nu, dt = 1.0 / c;
    const lattice_t L = lattice_of(p);
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k0 = cell(p, x, y, z);
                double rsum = 0.0, m[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < L.Q; ++i) {
                    int64_t km = cell(p, x - L.E[i][0], y - L.E[i][1], z - L.E[i][2]);
                    double um[3], Fm[3];
                    load3(u, N, km, um);
                    load3(F, N, km, Fm);
                    double fi = feq_c(&L, i, c, rho[km], um) + dt * fgzs_c(&L, i, c, um, Fm);
                    rsum += fi;
                    for (int a = 0; a < 3; ++a) m[a] += c * L.E[i][a] * fi;
                }
                rho_out[k0] = rsum;
                for (int a = 0; a < 3; ++a) u_out[a * N + k0] = (m[a] + 0.5 * dt * F[a * N + k0]) / rsum;
            }
}

/* One fluid update: the single-step predictor for tau < 1, the macroscopic branch for tau >= 1
 * (defined without rescaling only: gamma != 1 with tau >= 1 gives NaN). */
void orc_fluid(const orc_params *p, const double *rho, const double *u, const double *F,
               double *rho_out, double *u_out) {
    if (orc_fluid_tau(p) < 1.0) {
        fluid_single_step(p, rho, u, F, rho_out, u_out);
    } else if (gamma_of(p) == 1.0) {
        fluid_macroscopic(p, rho, u, F, rho_out, u_out);
    } else {
        const int64_t N = ncells(p);
        for (int64_t k = 0; k < N; ++k) rho_out[k] = NAN;
        for (int64_t k = 0; k < 3 * N; ++k) u_out[k] = NAN;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Flow rate over the pipe cross-section r <= R                                              */
/* ------------------------------------------------------------------------------------------ */
static void flow_sums(const orc_params *p, const double *u, double *sum_ux, int64_t *count) {
    double s = 0.0;
    int64_t n = 0;
    const double R2 = p->radius * p->radius;
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y) {
            double dy = y - p->yc, dz = z - p->zc;
            if (dy * dy + dz * dz > R2) continue;
            for (int x = 0; x < p->nx; ++x) {
                s += u[cell(p, x, y, z)];
                n++;
            }
        }
    *sum_ux = s;
    *count = n;
}

/* ------------------------------------------------------------------------------------------ */
/* Whole step                                                                                 */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    orc_params p;
    int64_t M;
    double *X, *uwall, *bwall, *d;
    double *bstar, *F, *rho2, *u2;
} orc_ctx;

orc_ctx *orc_create(const orc_params *p, int64_t M, const double *X, const double *uwall,
                    const double *bwall) {
    orc_ctx *c = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    c->p = *p;
    c->M = M;
    const int64_t N = ncells(p);
    if (M > 0) {
        c->X = (double *)malloc((size_t)(3 * M) * sizeof(double));
        memcpy(c->X, X, (size_t)(3 * M) * sizeof(double));
        c->d = (double *)malloc((size_t)M * sizeof(double));
        orc_ib_rowsums(p, M, X, c->d);
        if (uwall) {
            c->uwall = (double *)malloc((size_t)(3 * M) * sizeof(double));
            memcpy(c->uwall, uwall, (size_t)(3 * M) * sizeof(double));
        }
        if (bwall) {
            c->bwall = (double *)malloc((size_t)(3 * M) * sizeof(double));
            memcpy(c->bwall, bwall, (size_t)(3 * M) * sizeof(double));
        }
    }
    c->bstar = (double *)malloc((size_t)(3 * N) * sizeof(double));
    c->F = (double *)malloc((size_t)(3 * N) * sizeof(double));
    c->rho2 = (double *)malloc((size_t)N * sizeof(double));
    c->u2 = (double *)malloc((size_t)(3 * N) * sizeof(double));
    return c;
}

void orc_destroy(orc_ctx *c) {
    if (!c) return;
    free(c->X);
    free(c->uwall);
    free(c->bwall);
    free(c->d);
    free(c->bstar);
    free(c->F);
    free(c->rho2);
    free(c->u2);
    free(c);
}

void orc_get_rowsums(const orc_ctx *c, double *d) {
    if (c->M > 0) memcpy(d, c->d, (size_t)c->M * sizeof(double));
}

/* Resistivity ratio of the B correction: lambda_b <= 0 selects eta / eta_ref, eta_ref = 1/6. */
static double lambda_b_of(const orc_params *p) {
    return p->lambda_b > 0.0 ? p->lambda_b : p->eta * 6.0;
}

/* Advance n steps. t and G are the step counter and the (controlled) body force, in/out. */
void orc_step(orc_ctx *c, double *rho, double *u, double *b, int64_t n, int64_t *t, double *G) {
    const orc_params *p = &c->p;
    const int64_t N = ncells(p);
    const double PI = 3.14159265358979323846;
    for (int64_t s = 0; s < n; ++s) {
        double Gt;
        if (p->flow_control)
            Gt = *G;
        else if (p->period > 0.0)
            Gt = p->G0 + p->G1 * cos(2.0 * PI * (double)(*t) / p->period);
        else
            Gt = p->G0;
        /* 1. magnetic iteration with the wall correction after each sweep */
        for (int m = 0; m < p->n_mag; ++m) {
            orc_mag_sweep(p, u, b, c->bstar);
            if (p->ib_b && c->M > 0)
                orc_ib_correct(p, c->M, c->X, c->d, lambda_b_of(p), c->bwall, c->bstar);
            memcpy(b, c->bstar, (size_t)(3 * N) * sizeof(double));
        }
        /* 2. Lorentz + body force from the new b */
        orc_lorentz(p, b, Gt, c->F);
        /* 3. fluid predictor */
        orc_fluid(p, rho, u, c->F, c->rho2, c->u2);
        /* 4. velocity wall correction (density is not corrected) */
        if (p->ib_u && c->M > 0)
            orc_ib_correct(p, c->M, c->X, c->d, p->lambda_u > 0.0 ? p->lambda_u : 1.0, c->uwall, c->u2);
        memcpy(rho, c->rho2, (size_t)N * sizeof(double));
        memcpy(u, c->u2, (size_t)(3 * N) * sizeof(double));
        /* 5. flow-rate control of the driving force (integral law on the bulk velocity) */
        if (p->flow_control) {
            double sum;
            int64_t cnt;
            flow_sums(p, u, &sum, &cnt);
            double ub = cnt ? sum / (double)cnt : 0.0;
            *G = *G + p->k_c * (8.0 * p->nu / (p->radius * p->radius)) * (p->u_target - ub);
        } else {
            *G = Gt;
        }
        *t += 1;
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Energy budgets (Sec. 4): averages over Omega = {r < R_omega}, R_omega = omega_radius, or   */
/* R - 2 (inside the band the wall kernel touches) when omega_radius <= 0                     */
/* out[0..17] = E_k, E_m, E_b, P_in, P_p, P_nu, P_L, M_eta, M_adv, joule, mass, Q, u_max,       */
/*              n_omega, G, nonfinite, res_mag, D_eta                                         */
/* D_eta = -eta <b . lap b>: the Joule dissipation eta <|J|^2> written as the lattice Dirichlet */
/* form (equal to it for a divergence-free b that vanishes on the boundary of Omega), so that */
/* with -P_nu (the viscous dissipation in the same form) the steady power balance             */
/* P_in = -P_nu + D_eta closes over the conductor.                                            */
/* ------------------------------------------------------------------------------------------ */
void orc_budgets(const orc_params *p, const double *rho, const double *u, const double *b, double G,
                 double *out) {
    const int64_t N = ncells(p);
    double Ek = 0, Em = 0, Eb = 0, Pin = 0, Pp = 0, Pnu = 0, PL = 0, Meta = 0, Madv = 0, Jl = 0, Res = 0;
    double Deta = 0;
    double mass = 0, Q = 0, umax2 = 0;
    int64_t nom = 0;
    int nonfinite = 0;
    const double Ro = p->omega_radius > 0.0 ? p->omega_radius : p->radius - 2.0;
    const double Ro2 = Ro * Ro, R2 = p->radius * p->radius;
    double *prs = (double *)malloc((size_t)N * sizeof(double));
    double *lam = (double *)malloc((size_t)(9 * N) * sizeof(double)); /* Lambda_ac = u_c B_a - B_c u_a */
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k = cell(p, x, y, z);
                double B[3];
                orc_bext(p, x, y, z, B);
                for (int a = 0; a < 3; ++a) B[a] += b[a * N + k];
                prs[k] = CS2 * rho[k];
                for (int a = 0; a < 3; ++a)
                    for (int cc = 0; cc < 3; ++cc)
                        lam[(3 * a + cc) * N + k] = u[cc * N + k] * B[a] - B[cc] * u[a * N + k];
            }
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                int64_t k = cell(p, x, y, z);
                double uu[3], bb[3], B[3];
                load3(u, N, k, uu);
                load3(b, N, k, bb);
                orc_bext(p, x, y, z, B);
                for (int a = 0; a < 3; ++a) B[a] += bb[a];
                double u2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
                if (!isfinite(u2) || !isfinite(rho[k])) nonfinite = 1;
                if (u2 > umax2) umax2 = u2;
                mass += rho[k];
                double dy = y - p->yc, dz = z - p->zc, r2 = dy * dy + dz * dz;
                if (r2 <= R2) Q += uu[0];
                if (r2 >= Ro2) continue;
                nom++;
                double J[3], gp[3];
                curl_iso(p, b, x, y, z, J);
                grad_iso(p, prs, x, y, z, gp);
                double JxB[3] = {J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2],
                                 J[0] * B[1] - J[1] * B[0]};
                Ek += 0.5 * rho[k] * u2;
                Em += 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
                Eb += 0.5 * (bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2]);
                Pin += G * uu[0];
                for (int a = 0; a < 3; ++a) {
                    Pp += -uu[a] * gp[a];
                    Pnu += p->nu * uu[a] * lap_iso(p, u + a * N, x, y, z);
                    PL += uu[a] * JxB[a];
                    const double lapb = lap_iso(p, b + a * N, x, y, z);
                    Meta += p->eta * B[a] * lapb;
                    double div = 0.0;
                    for (int cc = 0; cc < 3; ++cc) {
                        double g[3];
                        grad_iso(p, lam + (3 * a + cc) * N, x, y, z, g);
                        div += g[cc];
                    }
                    Madv += -B[a] * div;
                    /* Sec. 5.8 eq. "Error l2 decay": eta lap b - div(u B - B u) */
                    Res += (p->eta * lapb - div) * (p->eta * lapb - div);
                    Jl += p->eta * J[a] * J[a];
                    Deta += -p->eta * bb[a] * lapb;
                }
            }
    free(prs);
    free(lam);
    double inv = nom ? 1.0 / (double)nom : 0.0;
    out[0] = Ek * inv;
    out[1] = Em * inv;
    out[2] = Eb * inv;
    out[3] = Pin * inv;
    out[4] = Pp * inv;
    out[5] = Pnu * inv;
    out[6] = PL * inv;
    out[7] = Meta * inv;
    out[8] = Madv * inv;
    out[9] = Jl * inv;
    out[10] = mass;
    out[11] = Q / (double)p->nx;
    out[12] = sqrt(umax2);
    out[13] = (double)nom;
    out[14] = G;
    out[15] = (double)nonfinite;
    out[16] = sqrt(Res * inv); /* root mean square over Omega of the induction residual */
    out[17] = Deta * inv;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
