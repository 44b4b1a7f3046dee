// Host runtime of mhdlbm: workspace carving, argument checks, marker preprocessing (Lagrange
// taps, row sums d_j, gather lists), the step launch sequence and the C ABI of include/mhdlbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "mhd_internal.h"

using namespace mhd;

// The Python binding mirrors these structs field by field (tests check the same sizes).
static_assert(sizeof(mhd_grid_desc) == 40, "mhd_grid_desc layout");
static_assert(sizeof(mhd_params) == 176, "mhd_params layout");
static_assert(sizeof(mhd_budget) == 144, "mhd_budget layout");
static_assert(sizeof(mhd_pipe_desc) == 48, "mhd_pipe_desc layout");

namespace {

thread_local std::string g_err;

mhd_status fail(mhd_status st, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
mhd_status fail(mhd_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail(MHD_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t kind_bytes(int k) { return k == MHD_STORE_F32 ? 4 : 2; }
bool is_split(const mhd_grid_desc &g) { return g.b_storage == MHD_STORE_F16_SPLIT; }

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Padded gather entries reserved per marker of capacity (band cells x entries per cell).
constexpr int64_t kBandSlots = 64;

// Byte offsets of every region of the caller's workspace.
struct Layout {
    size_t rho[2], u[2], b[2], bh[2], u16, F, bext, bext_yz, ctrl, tap_cell, tap_w, s_u, s_b, uwall, bwall, delta;
    size_t band_cell, band_mk, band_w, red_part, flow_part, ring, res, total;
    size_t ring_tap, ring_tw, row_off, row_mk, row_w;  // line-structured walls
};

Layout make_layout(const mhd_grid_desc &g, int64_t M) {
    Layout L{};
    const int64_t N = (int64_t)g.nx * g.ny * g.nz;
    const int64_t T = 27 * std::max<int64_t>(M, 0);  // taps, at most 27 per marker
    const int64_t TB = kBandSlots * std::max<int64_t>(M, 0);  // padded gather entries
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    for (int i = 0; i < 2; ++i) L.rho[i] = take(N * kind_bytes(g.rho_storage));
    for (int i = 0; i < 2; ++i) L.u[i] = take(3 * N * kind_bytes(g.u_storage));
    for (int i = 0; i < 2; ++i) L.b[i] = take(3 * N * kind_bytes(g.b_storage));
    if (is_split(g)) {  // hi parts of b and the float16 copy of u
        for (int i = 0; i < 2; ++i) L.bh[i] = take(3 * N * 2);
        L.u16 = take(3 * N * 2);
    }
    L.F = take(3 * N * sizeof(float));
    L.bext = take(3 * (size_t)g.nx * sizeof(float));
    L.bext_yz = take(3 * (size_t)g.ny * g.nz * sizeof(float));
    L.ctrl = take(sizeof(DevCtrl));
    L.tap_cell = take(T * sizeof(int));
    L.tap_w = take(T * sizeof(float));
    L.s_u = take(M * sizeof(float));
    L.s_b = take(M * sizeof(float));
    L.uwall = take(3 * M * sizeof(float));
    L.bwall = take(3 * M * sizeof(float));
    L.delta = take(3 * M * sizeof(float));
    L.band_cell = take(T * sizeof(int));
    L.band_mk = take(TB * sizeof(int));
    L.band_w = take(TB * sizeof(float));
    // line tables: lines * taps, band rows and rows * entries are each at most M when n_x >= 64
    L.ring_tap = take(M * sizeof(int));
    L.ring_tw = take(M * sizeof(float));
    L.row_off = take(M * sizeof(int));
    L.row_mk = take(M * sizeof(int));
    L.row_w = take(M * sizeof(float));
    L.red_part = take((size_t)kRedBlocks * kBudgetVals * sizeof(double));
    L.flow_part = take((size_t)kRedBlocks * sizeof(double));
    L.ring = take((size_t)kRingCap * sizeof(mhd_budget));
    L.res = take((size_t)kResCap * sizeof(double));
    L.total = off;
    return L;
}

mhd_status check_desc(const mhd_grid_desc *g) {
    if (!g) return fail(MHD_ERR_INVALID_ARG, "grid descriptor is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(MHD_ERR_INVALID_ARG, "box size must be >= 1 per axis");
    const int64_t N = (int64_t)g->nx * g->ny * g->nz;
    if (3 * N >= (int64_t)1 << 31) return fail(MHD_ERR_INVALID_ARG, "3*nx*ny*nz must stay below 2^31");
    for (int k : {g->rho_storage, g->u_storage, g->b_storage})
        if (k < MHD_STORE_F32 || k > MHD_STORE_F16_SPLIT) return fail(MHD_ERR_INVALID_ARG, "unknown storage kind %d", k);
    const int r = g->rho_storage, u = g->u_storage, b = g->b_storage;
    const bool ok = (r == 0 && u == 0 && b == 0) || (r == 1 && u == 1 && b == 1) || (r == 1 && u == 2 && b == 1) ||
                    (r == 2 && u == 2 && b == 2) || (r == 0 && u == 0 && b == 3);
    if (!ok)
        return fail(MHD_ERR_UNSUPPORTED,
                    "storage mix (rho %d, u %d, b %d) not built: use all f32, f16/f16/f16, f16/bf16/f16, all bf16 or "
                    "f32/f32/f16-split", r, u, b);
    if ((u != 0 || b == 3) && !(g->u_scale > 0.0)) return fail(MHD_ERR_INVALID_ARG, "u_scale must be > 0 for 16-bit u");
    if (b != 0 && !(g->b_scale > 0.0)) return fail(MHD_ERR_INVALID_ARG, "b_scale must be > 0 for 16-bit b");
    return MHD_OK;
}

// Three-point Lagrange weights of the nodes n0-1, n0, n0+1 nearest to X (n0 = floor(X + 1/2),
// s = X - n0 in [-1/2, 1/2)): the quadratic through the three nodes evaluated at X.
inline int lagrange_nodes(double X, double w[3]) {
    const int n0 = (int)std::floor(X + 0.5);
    const double s = X - n0;
    w[0] = -0.5 * s * (1.0 - s);
    w[1] = 1.0 - s * s;
    w[2] = 0.5 * s * (1.0 + s);
    return n0 - 1;
}

inline int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

struct Event2 {
    hipEvent_t a, b;
};

}  // namespace

struct mhd_sim {
    mhd_grid_desc g{};
    int64_t N = 0, Mcap = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    char *ws = nullptr;
    Layout L{};
    int kinds = 0;
    // ping-pong state (ch: hi part of b in the split form)
    int cr = 0, cu = 0, cb = 0, ch = 0;
    // host state
    bool have_params = false;
    mhd_params prm{};
    int64_t M = 0, nband = 0;
    int tm = 0, km = 0;
    std::vector<double> d;  // row sums of D D^T (internal marker order)
    // line-structured wall (tables uploaded) and whether its kernels are used (MHD_IB_RING=0: the
    // general tables, same bits)
    bool lines = false, ring_on = false;
    int64_t t_host = 0;
    SweepLaunch sweep{64, 4, 8, 0};
    double flow_inv_count = 0.0;
    // profiling
    bool prof = false;
    std::vector<Event2> ev_pool[MHD_K_COUNT];
    size_t ev_used[MHD_K_COUNT] = {};
    mhd_batch *owner = nullptr;  // batch this box belongs to (it then owns the box)
    // Step graphs: one fluid step captured per state of the double buffers and replayed (only on
    // a caller stream; dropped whenever parameters, markers or tiles change).
    struct StepGraph {
        int key;                 // buffer state before the step
        int cb, cr, cu, ch;      // buffer state after it
        hipGraphExec_t exec;
    };
    std::vector<StepGraph> graphs;
    bool graph_on = true;
    bool fused_lf = true;  // Lorentz + fluid in one launch where the storage allows (MHD_FUSED_LF=0: two)
    // Scratch of the step kernels taken from elsewhere than the workspace while set (the
    // allocation-free entry point): Lorentz force F, wall corrections, flow and budget partials.
    struct Scratch {
        float *F = nullptr, *delta = nullptr;
        double *flow = nullptr, *red = nullptr;
    } scr;

    template <typename T>
    T *at(size_t off) const {
        return reinterpret_cast<T *>(ws + off);
    }
    void *rho(int i) const { return ws + L.rho[i]; }
    void *u(int i) const { return ws + L.u[i]; }
    void *b(int i) const { return ws + L.b[i]; }
    bool split() const { return g.b_storage == MHD_STORE_F16_SPLIT; }
    void *bh(int i) const { return split() ? ws + L.bh[i] : nullptr; }
    void *u16() const { return split() ? ws + L.u16 : nullptr; }
    const float *byz() const {  // (y, z) part of B_ext, present for the six-magnet field only
        return have_params && prm.bext_kind == MHD_BEXT_SIX_MAGNETS ? reinterpret_cast<const float *>(ws + L.bext_yz)
                                                                    : nullptr;
    }
    DevCtrl *ctrl() const { return at<DevCtrl>(L.ctrl); }
    float *F_buf() const { return scr.F ? scr.F : at<float>(L.F); }
    float *delta_buf() const { return scr.delta ? scr.delta : at<float>(L.delta); }
    double *flow_buf() const { return scr.flow ? scr.flow : at<double>(L.flow_part); }
    double *red_buf() const { return scr.red ? scr.red : at<double>(L.red_part); }
};

namespace {

void batch_touch(mhd_batch *b);  // the launch plan of a batch must be rebuilt

// The captured steps bake in parameters, marker tables and tiles: drop them on any change.
void drop_step_graphs(mhd_sim *s) {
    if (s->graphs.empty()) return;
    (void)hipStreamSynchronize(s->stream);
    for (auto &g : s->graphs) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
}

double gamma_of(const mhd_params &p) { return p.gamma > 0.0 ? p.gamma : 1.0; }
// tau = 3 nu / gamma + 1/2 >= 1: the macroscopic branch (set_params admits it with gamma = 1 only)
bool fluid_branch_mac(const mhd_params &p) { return !(3.0 * p.nu / gamma_of(p) + 0.5 < 1.0); }

StepConst step_const(const mhd_sim *s) {
    StepConst c{};
    c.nx = s->g.nx;
    c.ny = s->g.ny;
    c.nz = s->g.nz;
    const mhd_params &p = s->prm;
    c.kappa = (float)(1.0 / (2.0 * p.eta));
    const double gamma = gamma_of(p);
    c.tau = (float)(3.0 * p.nu / gamma + 0.5);
    c.inv_gamma = (float)(1.0 / gamma);
    c.mac = fluid_branch_mac(p) ? 1 : 0;
    c.mac_c = (float)(6.0 * p.nu);
    c.inv_mac_c = (float)(1.0 / (6.0 * p.nu));
    c.u_limit2 = c.mac ? 12.0 * p.nu * p.nu : 1.0 / 3.0;
    c.status = &s->ctrl()->status;
    c.u_scale = s->g.u_storage == MHD_STORE_F32 ? 1.0f : (float)s->g.u_scale;
    c.inv_u_scale = s->g.u_storage == MHD_STORE_F32 ? 1.0f : (float)(1.0 / s->g.u_scale);
    c.b_scale = s->g.b_storage == MHD_STORE_F32 ? 1.0f : (float)s->g.b_scale;
    c.inv_b_scale = s->g.b_storage == MHD_STORE_F32 ? 1.0f : (float)(1.0 / s->g.b_scale);
    c.omega = (float)(1.0 / (p.alpha > 0.0 ? p.alpha : 1.0));
    c.lattice = p.lattice == 27 ? 27 : 19;
    c.copy_scale = s->split() ? (float)s->g.u_scale : 1.0f;
    c.inv_copy_scale = s->split() ? (float)(1.0 / s->g.u_scale) : 1.0f;
    c.nu = p.nu;
    c.eta = p.eta;
    c.G0 = p.G0;
    c.G1 = p.G1;
    c.period = p.period;
    c.yc = p.yc;
    c.zc = p.zc;
    c.radius = p.avg_radius;
    c.omega_radius = p.omega_radius > 0.0 ? p.omega_radius : p.avg_radius - 2.0;
    c.flow_control = p.flow_control;
    c.u_target = p.u_bulk_target;
    c.k_c = p.k_c;
    return c;
}

double lambda_u_of(const mhd_params &p) { return p.lambda_u > 0.0 ? p.lambda_u : 1.0; }
double lambda_b_of(const mhd_params &p) { return p.lambda_b > 0.0 ? p.lambda_b : 6.0 * p.eta; }

// s_j = lambda / (d_j (1 + d_j (lambda - 1))) for both fields, uploaded to the workspace.
mhd_status upload_scalings(mhd_sim *s) {
    if (!s->have_params || s->M == 0) return MHD_OK;
    const double lu = lambda_u_of(s->prm), lb = lambda_b_of(s->prm);
    std::vector<float> su(s->M), sb(s->M);
    for (int64_t j = 0; j < s->M; ++j) {
        const double dj = s->d[j];
        const double qu = 1.0 + dj * (lu - 1.0), qb = 1.0 + dj * (lb - 1.0);
        if (!(dj > 0.0) || !(qu > 0.0) || !(qb > 0.0))
            return fail(MHD_ERR_INVALID_ARG,
                        "marker %lld: d_j = %g makes the wall scaling singular (1 + d (lambda - 1) = %g / %g)",
                        (long long)j, dj, qu, qb);
        su[j] = (float)(lu / (dj * qu));
        sb[j] = (float)(lb / (dj * qb));
    }
    HIPCHK(hipMemcpyAsync(s->at<float>(s->L.s_u), su.data(), s->M * sizeof(float), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->at<float>(s->L.s_b), sb.data(), s->M * sizeof(float), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return MHD_OK;
}

// Six magnets with alternating poles on a hexagon around (yc, zc) (Sec. 6): the (y, z) field
// of magnet k (angle 60 k degrees, strip of half-width Lh tangential, local z' radial outwards,
// polarity (-1)^k), summed; unscaled.
void hexapole_field(const mhd_params &p, double Lh, double D, double y, double z, double &By, double &Bz) {
    By = Bz = 0.0;
    for (int k = 0; k < 6; ++k) {
        const double ang = k * (3.14159265358979323846 / 3.0);
        const double ny_ = std::cos(ang), nz_ = std::sin(ang);  // radial unit vector
        const double ty = -nz_, tz = ny_;                          // tangential unit vector
        const double dy = y - (p.yc + D * ny_), dz = z - (p.zc + D * nz_);
        const double yl = dy * ty + dz * tz, zl = dy * ny_ + dz * nz_;
        const double fy = 2.0 * (std::atan((yl - Lh) / zl) - std::atan((yl + Lh) / zl));
        const double fz = std::log(((yl + Lh) * (yl + Lh) + zl * zl) / ((yl - Lh) * (yl - Lh) + zl * zl));
        const double sign = (k & 1) ? -1.0 : 1.0;
        By += sign * (fy * ty + fz * ny_);
        Bz += sign * (fy * tz + fz * nz_);
    }
}

// Imposed field: per x plane (3 x nx table) and, for the six magnets, per (y, z) (3 x ny nz).
mhd_status upload_bext(mhd_sim *s) {
    const int nx = s->g.nx, ny = s->g.ny, nz = s->g.nz;
    std::vector<float> t(3 * (size_t)nx, 0.f);
    const mhd_params &p = s->prm;
    for (int x = 0; x < nx; ++x) {
        double By = 0.0;
        if (p.bext_kind == MHD_BEXT_UNIFORM_Y)
            By = p.B0;
        else if (p.bext_kind == MHD_BEXT_TANH_FRINGE_Y)
            By = p.B0 * 0.5 * (1.0 + std::tanh(((double)x - p.fringe_x0) / p.fringe_w));
        t[nx + x] = (float)By;
    }
    HIPCHK(hipMemcpyAsync(s->at<float>(s->L.bext), t.data(), t.size() * sizeof(float), hipMemcpyHostToDevice,
                          s->stream));
    if (p.bext_kind == MHD_BEXT_SIX_MAGNETS) {
        const double Lh = p.magnet_half_width > 0.0 ? p.magnet_half_width : p.avg_radius / 6.0;
        double D = p.magnet_distance;
        if (!(D > 0.0)) {  // beyond the farthest cell of the box
            const double fy = std::max(p.yc, (double)(ny - 1) - p.yc), fz = std::max(p.zc, (double)(nz - 1) - p.zc);
            D = std::sqrt(fy * fy + fz * fz) + Lh + 1.0;
        }
        double ry, rz;
        hexapole_field(p, Lh, D, p.yc + p.avg_radius, p.zc, ry, rz);
        const double scale = p.B0 / std::sqrt(ry * ry + rz * rz);
        const size_t pyz = (size_t)ny * nz;
        std::vector<float> tyz(3 * pyz, 0.f);
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y) {
                double By, Bz;
                hexapole_field(p, Lh, D, (double)y, (double)z, By, Bz);
                if (!std::isfinite(By) || !std::isfinite(Bz))
                    return fail(MHD_ERR_INVALID_ARG, "six-magnet field is singular at cell (y %d, z %d): magnets inside the box",
                                y, z);
                tyz[pyz + y + (size_t)ny * z] = (float)(scale * By);
                tyz[2 * pyz + y + (size_t)ny * z] = (float)(scale * Bz);
            }
        HIPCHK(hipMemcpyAsync(s->at<float>(s->L.bext_yz), tyz.data(), tyz.size() * sizeof(float), hipMemcpyHostToDevice,
                              s->stream));
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return MHD_OK;
}

mhd_status fill_field(mhd_sim *s, mhd_field f, const double *host, bool zero) {
    const int64_t N = s->N;
    const int ncomp = f == MHD_FIELD_RHO ? 1 : 3;
    const int64_t n = ncomp * N;
    int kind;
    double scale = 1.0, offset = 0.0;
    void *dst;
    if (f == MHD_FIELD_RHO) {
        kind = s->g.rho_storage;
        offset = 1.0;
        dst = s->rho(s->cr);
    } else if (f == MHD_FIELD_U) {
        kind = s->g.u_storage;
        if (kind != MHD_STORE_F32) scale = s->g.u_scale;
        dst = s->u(s->cu);
    } else {
        kind = s->g.b_storage;
        if (kind != MHD_STORE_F32) scale = s->g.b_scale;
        dst = s->b(s->cb);
    }
    std::vector<float> tmp((size_t)n);
    for (int64_t i = 0; i < n; ++i) tmp[i] = zero ? 0.f : (float)((host[i] - offset) / scale);
    float *stage = s->at<float>(s->L.F);  // 3N floats, free between steps
    HIPCHK(hipMemcpyAsync(stage, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, s->stream));
    if (f == MHD_FIELD_B_INDUCED && s->split()) {
        HIPCHK(launch_store_split(s->stream, stage, s->bh(s->ch), dst, n));
    } else {
        HIPCHK(launch_store_kind(s->stream, kind, stage, dst, n));
    }
    if (f == MHD_FIELD_U && s->split()) {  // float16 copy u / u_scale read by the sweeps
        HIPCHK(hipStreamSynchronize(s->stream));
        const double inv = 1.0 / s->g.u_scale;
        for (int64_t i = 0; i < n; ++i) tmp[i] = zero ? 0.f : (float)(host[i] * inv);
        HIPCHK(hipMemcpyAsync(stage, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, s->stream));
        HIPCHK(launch_store_kind(s->stream, MHD_STORE_F16, stage, s->u16(), n));
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    return MHD_OK;
}

inline Event2 &next_event(mhd_sim *s, int k) {
    if (s->ev_used[k] == s->ev_pool[k].size()) {
        Event2 e;
        (void)hipEventCreate(&e.a);
        (void)hipEventCreate(&e.b);
        s->ev_pool[k].push_back(e);
    }
    return s->ev_pool[k][s->ev_used[k]++];
}

// Launch helper: brackets the launch with events when profiling is on.
template <typename Fn>
mhd_status timed(mhd_sim *s, int k, const char *what, Fn fn) {
    Event2 *e = nullptr;
    if (s->prof) {
        e = &next_event(s, k);
        HIPCHK(hipEventRecord(e->a, s->stream));
    }
    hipError_t err = fn();
    if (err != hipSuccess) return fail(MHD_ERR_HIP, "launch of %s failed: %s", what, hipGetErrorString(err));
    if (e) HIPCHK(hipEventRecord(e->b, s->stream));
    return MHD_OK;
}

#define STEPCHK(x)                     \
    do {                               \
        mhd_status st_ = (x);          \
        if (st_ != MHD_OK) return st_; \
    } while (0)

IbArgs ib_args(mhd_sim *s, const float *sj, const float *wall);

mhd_status ib_correct(mhd_sim *s, int kind, void *phi, float scale, float inv_scale, const float *sj,
                      const float *wall, const void *phi_hi, void *copy, float copy_inv) {
    if (s->M == 0) return MHD_OK;
    IbArgs a = ib_args(s, sj, wall);
    a.phi_hi = phi_hi;
    a.copy = copy;
    a.copy_inv = copy_inv;
    a.delta = s->delta_buf();
    return timed(s, MHD_K_IB, "wall correction",
                 [&] { return launch_ib(s->stream, kind, phi, scale, inv_scale, a); });
}

// Magnetic sweep m of a fluid step (m = 0 re-splits the split form) and its b wall correction.
mhd_status mag_iteration(mhd_sim *s, const StepConst &c, int m) {
    hipStream_t st = s->stream;
    {
        const int nb = 1 - s->cb;
        {  // timed by events the launch stamps at kernel start / end
            SweepArgs a = make_sweep_args(s->split() ? s->u16() : s->u(s->cu), s->b(s->cb), s->b(nb),
                                          s->at<float>(s->L.bext), c, s->sweep);
            a.bext_yz = s->byz();
            if (s->split()) {  // first sweep of the step re-splits b into a new hi and lo
                a.u_scale = c.copy_scale;
                a.bh = s->bh(s->ch);
                if (m == 0) a.bho = s->bh(1 - s->ch);
            }
            Event2 *e = s->prof ? &next_event(s, MHD_K_MAG_SWEEP) : nullptr;
            const hipError_t err = launch_mag_sweep(st, s->kinds, a, s->sweep, e ? e->a : nullptr, e ? e->b : nullptr);
            if (err != hipSuccess) return fail(MHD_ERR_HIP, "launch of mag_sweep failed: %s", hipGetErrorString(err));
            if (s->split() && m == 0) s->ch = 1 - s->ch;
        }
        STEPCHK(ib_correct(s, s->g.b_storage, s->b(nb), c.b_scale, c.inv_b_scale, s->at<float>(s->L.s_b),
                           s->at<float>(s->L.bwall), s->bh(s->ch), nullptr, 0.f));
        s->cb = nb;
    }
    return MHD_OK;
}

mhd_status one_step(mhd_sim *s) {
    const StepConst c = step_const(s);
    hipStream_t st = s->stream;
    STEPCHK(timed(s, MHD_K_CONTROL, "ctrl_begin", [&] { return launch_ctrl_begin(st, s->ctrl(), c); }));
    // 1. magnetic iteration, wall correction after every sweep
    for (int m = 0; m < s->prm.n_mag; ++m) STEPCHK(mag_iteration(s, c, m));
    // 2. Lorentz + body force from the new b, 3. fluid predictor (one launch for float32 boxes:
    // the force then stays in LDS), 4. velocity wall correction
    const int nr = 1 - s->cr, nu = 1 - s->cu;
    if (s->fused_lf && s->kinds == pack_kinds(MHD_STORE_F32, MHD_STORE_F32, MHD_STORE_F32)) {
        LfArgs a{};
        a.rho = static_cast<const float *>(s->rho(s->cr));
        a.u = static_cast<const float *>(s->u(s->cu));
        a.b = static_cast<const float *>(s->b(s->cb));
        a.bext = s->at<float>(s->L.bext);
        a.bext_yz = s->byz();
        a.ctrl = s->ctrl();
        a.rho_o = static_cast<float *>(s->rho(nr));
        a.u_o = static_cast<float *>(s->u(nu));
        a.c = c;
        STEPCHK(timed(s, MHD_K_FLUID, "lorentz + fluid", [&] { return launch_lorentz_fluid(st, a); }));
    } else {
        float *F = s->F_buf();
        STEPCHK(timed(s, MHD_K_LORENTZ, "lorentz", [&] {
            return launch_lorentz(st, s->g.b_storage, s->b(s->cb), s->bh(s->ch), s->at<float>(s->L.bext), s->byz(),
                                  s->ctrl(), F, c);
        }));
        STEPCHK(timed(s, MHD_K_FLUID, "fluid", [&] {
            return launch_fluid(st, s->kinds, s->rho(s->cr), s->u(s->cu), F, s->rho(nr), s->u(nu), s->u16(), c);
        }));
    }
    STEPCHK(ib_correct(s, s->g.u_storage, s->u(nu), c.u_scale, c.inv_u_scale, s->at<float>(s->L.s_u),
                       s->at<float>(s->L.uwall), nullptr, s->u16(), c.inv_copy_scale));
    s->cr = nr;
    s->cu = nu;
    // 5. flow-rate control sum (float64, fixed order) and step counter
    double *fp = s->flow_buf();
    if (c.flow_control)
        STEPCHK(timed(s, MHD_K_CONTROL, "flow_partial",
                      [&] { return launch_flow_partial(st, s->g.u_storage, s->u(s->cu), fp, c); }));
    STEPCHK(timed(s, MHD_K_CONTROL, "step_end",
                  [&] { return launch_step_end(st, s->ctrl(), fp, c, s->flow_inv_count); }));
    s->t_host += 1;
    return MHD_OK;
}

mhd_status record_budget(mhd_sim *s) {
    const StepConst c = step_const(s);
    return timed(s, MHD_K_BUDGET, "budget", [&] {
        return launch_budget(s->stream, s->kinds, s->rho(s->cr), s->u(s->cu), s->b(s->cb), s->bh(s->ch),
                             s->at<float>(s->L.bext), s->byz(), s->ctrl(), s->red_buf(),
                             s->at<mhd_budget>(s->L.ring), c);
    });
}

mhd_status read_ctrl(mhd_sim *s, DevCtrl *h) {
    HIPCHK(hipMemcpyAsync(h, s->ctrl(), sizeof(DevCtrl), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return MHD_OK;
}

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

bool valid_tx(int tx) { return tx == 8 || tx == 16 || tx == 32 || tx == 64; }

// Workgroups of one sweep launch with tiles L on an nx x ny x nz box.
int64_t sweep_workgroups(const SweepLaunch &L, int nx, int ny, int nz) {
    const bool pair = L.pair && nx % 128 == 0;
    const int64_t tx = pair ? 128 : L.tx, ty = pair ? (L.ty >= 8 ? 8 : 4) : 256 / L.tx;
    return ((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + L.zchunk - 1) / L.zchunk);
}

// Default sweep tiles of a box (environment overrides for experiments: MHD_SWEEP_TX,
// MHD_SWEEP_ZCHUNK, MHD_SWEEP_PAIR, MHD_SWEEP_PAIR_TY). Each z chunk re-reads two halo planes,
// which costs HBM traffic on large boxes, while small boxes need short chunks for enough
// workgroups. The chunk is the longest of 64, 32, 16 planes that still gives 512 workgroups
// (two per CU) for the paired float32 sweep, 2048 for the other forms, else 8 planes. Measured
// per sweep: 512 x 256^2 float32 353 -> 283 us (64 planes; 272 us with 8-row tiles), split
// form 282 -> 252 us (32); 256^3 171 -> 140 us (64; 136 us with 8 rows); 200^3 single-cell
// tiles 102 -> 96 us (16); 128^3 stays at 8 planes and 4 rows (19 us; 16 planes, one
// workgroup per CU: 26 us; 8 rows: 20 us).
SweepLaunch default_tiles(const mhd_grid_desc &g) {
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    SweepLaunch L;
    L.tx = nx >= 64 ? 64 : nx >= 32 ? 32 : nx >= 16 ? 16 : 8;
    const int etx = env_int("MHD_SWEEP_TX", L.tx);
    if (valid_tx(etx)) L.tx = etx;
    L.pair = (nx % 128 == 0) && env_int("MHD_SWEEP_PAIR", 1) != 0;
    L.ty = env_int("MHD_SWEEP_PAIR_TY", 4) >= 8 ? 8 : 4;
    L.zchunk = 8;
    const bool plain_pair = L.pair && g.b_storage == MHD_STORE_F32 && g.u_storage == MHD_STORE_F32;
    const int64_t need = plain_pair ? 512 : 2048;
    for (int zc : {64, 32, 16}) {
        SweepLaunch t = L;
        t.zchunk = zc;
        if (sweep_workgroups(t, nx, ny, nz) >= need) {
            L.zchunk = zc;
            break;
        }
    }
    // long chunks of the paired float32 sweep: 8-row tiles when that still leaves 256
    // workgroups (the same 2048 waves); 2-4% shorter sweeps on 128 x 256^2 to 512 x 256^2 boxes.
    // An 8-row workgroup of the float32 sweep holds a CU's register file alone (150-170 VGPRs,
    // two waves per SIMD), so 256 workgroups run in one round: the chunk then doubles up to 128
    // planes while 256 remain (512 x 256^2: 272-273 -> 265 us, half the halo planes).
    if (plain_pair && L.zchunk >= 32 && env_int("MHD_SWEEP_PAIR_TY", 0) == 0) {
        SweepLaunch t = L;
        t.ty = 8;
        if (sweep_workgroups(t, nx, ny, nz) >= 256) {
            L.ty = 8;
            for (t.zchunk = 2 * L.zchunk; t.zchunk <= 128 && sweep_workgroups(t, nx, ny, nz) >= 256; t.zchunk *= 2)
                L.zchunk = t.zchunk;
        }
    }
    L.zchunk = std::max(1, env_int("MHD_SWEEP_ZCHUNK", L.zchunk));
    return L;
}

// The tile choice a launch really uses (the paired form needs nx % 128 == 0).
SweepLaunch effective_tiles(const SweepLaunch &L, int nx) {
    SweepLaunch e = L;
    e.pair = L.pair && nx % 128 == 0;
    e.ty = L.ty >= 8 ? 8 : 4;
    return e;
}

}  // namespace

extern "C" {

const char *mhd_last_error(void) { return g_err.c_str(); }

mhd_status mhd_workspace_size(const mhd_grid_desc *g, int64_t n_markers, size_t *bytes) {
    g_err.clear();
    STEPCHK(check_desc(g));
    if (!bytes) return fail(MHD_ERR_INVALID_ARG, "bytes is NULL");
    if (n_markers < 0 || n_markers >= ((int64_t)1 << 26))
        return fail(MHD_ERR_INVALID_ARG, "n_markers must be in [0, 2^26)");
    *bytes = make_layout(*g, n_markers).total;
    return MHD_OK;
}

mhd_status mhd_create(const mhd_grid_desc *g, int64_t n_markers, void *dev_workspace, size_t bytes, void *hip_stream,
                      mhd_sim **out) {
    g_err.clear();
    if (!out) return fail(MHD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    STEPCHK(check_desc(g));
    if (n_markers < 0 || n_markers >= ((int64_t)1 << 26))
        return fail(MHD_ERR_INVALID_ARG, "n_markers must be in [0, 2^26)");
    if (!dev_workspace) return fail(MHD_ERR_INVALID_ARG, "device workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256) return fail(MHD_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    const Layout L = make_layout(*g, n_markers);
    if (bytes < L.total)
        return fail(MHD_ERR_OOM, "workspace has %zu bytes, %zu needed", bytes, L.total);
    mhd_sim *s = new (std::nothrow) mhd_sim();
    if (!s) return fail(MHD_ERR_OOM, "host allocation failed");
    s->g = *g;
    s->N = (int64_t)g->nx * g->ny * g->nz;
    s->Mcap = n_markers;
    s->stream = reinterpret_cast<hipStream_t>(hip_stream);
    s->ws = static_cast<char *>(dev_workspace);
    s->L = L;
    s->kinds = pack_kinds(g->rho_storage, g->u_storage, g->b_storage);
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return fail(MHD_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    }
    // tile shape: widest x tile that the box fills, 256 work-items per workgroup; two x cells
    // per lane whenever a row splits into 128-cell tiles (fewer LDS reads per cell); z chunk by
    // box size
    s->sweep = default_tiles(*g);
    // initial state: rho = 1, u = 0, b = 0, t = 0, G = 0
    DevCtrl hc{};
    auto cleanup = [&](mhd_status r) {
        delete s;
        return r;
    };
    e = hipMemsetAsync(s->ws, 0, L.total, s->stream);
    if (e != hipSuccess) return cleanup(fail(MHD_ERR_HIP, "hipMemsetAsync failed: %s", hipGetErrorString(e)));
    e = hipMemcpyAsync(s->ctrl(), &hc, sizeof hc, hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return cleanup(fail(MHD_ERR_HIP, "hipMemcpyAsync failed: %s", hipGetErrorString(e)));
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return cleanup(fail(MHD_ERR_HIP, "hipStreamSynchronize failed: %s", hipGetErrorString(e)));
    *out = s;
    return MHD_OK;
}

mhd_status mhd_set_markers(mhd_sim *s, const double *xyz, int64_t M, const double *u_wall, const double *b_wall) {
    g_err.clear();
    if (!s) return fail(MHD_ERR_INVALID_ARG, "sim is NULL");
    drop_step_graphs(s);
    if (M < 0 || M > s->Mcap) return fail(MHD_ERR_INVALID_ARG, "M = %lld outside [0, %lld]", (long long)M, (long long)s->Mcap);
    if (M > 0 && !xyz) return fail(MHD_ERR_INVALID_ARG, "xyz is NULL");
    const int n[3] = {s->g.nx, s->g.ny, s->g.nz};
    for (int64_t j = 0; j < M; ++j)
        for (int a = 0; a < 3; ++a) {
            const double v = xyz[a * M + j];
            if (!(v >= 0.0 && v < (double)n[a]))
                return fail(MHD_ERR_INVALID_ARG, "marker %lld coordinate %d = %g outside [0, %d)", (long long)j, a, v, n[a]);
        }
    // 1. nonzero Lagrange taps of every marker (original order)
    std::vector<int> tptr((size_t)M + 1, 0), tcell;
    std::vector<double> tw;
    tcell.reserve((size_t)M * 9);
    tw.reserve((size_t)M * 9);
    for (int64_t j = 0; j < M; ++j) {
        double w[3][3];
        int base[3];
        for (int a = 0; a < 3; ++a) base[a] = lagrange_nodes(xyz[a * M + j], w[a]);
        for (int cz = 0; cz < 3; ++cz)
            for (int cy = 0; cy < 3; ++cy)
                for (int cx = 0; cx < 3; ++cx) {
                    const double wt = w[0][cx] * w[1][cy] * w[2][cz];
                    if (wt == 0.0) continue;
                    const int64_t k = wrap(base[0] + cx, n[0]) +
                                      (int64_t)n[0] * (wrap(base[1] + cy, n[1]) + (int64_t)n[1] * wrap(base[2] + cz, n[2]));
                    tcell.push_back((int)k);
                    tw.push_back(wt);
                }
        tptr[j + 1] = (int)tcell.size();
    }
    // 2. row sums d_j = sum_k D_jk (sum_i D_ik): the taps grouped by cell with a stable sort
    //    (each cell's weights summed in tap order), the cell sum handed back to every tap
    const size_t T = tcell.size();
    std::vector<double> d0((size_t)M);
    {
        std::vector<uint32_t> ord(T);
        for (size_t t = 0; t < T; ++t) ord[t] = (uint32_t)t;
        std::stable_sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return tcell[a] < tcell[b]; });
        std::vector<double> Stap(T);
        for (size_t a = 0; a < T;) {
            size_t b = a;
            double acc = 0.0;
            while (b < T && tcell[ord[b]] == tcell[ord[a]]) acc += tw[ord[b++]];
            for (size_t k = a; k < b; ++k) Stap[ord[k]] = acc;
            a = b;
        }
        for (int64_t j = 0; j < M; ++j) {
            double acc = 0.0;
            for (int t = tptr[j]; t < tptr[j + 1]; ++t) acc += tw[t] * Stap[t];
            d0[j] = acc;
        }
    }
    // 3. internal order: by the (y, z) of the first tap, then x, so that markers at the same
    //    cross-section position on neighbouring x planes sit next to each other. Line-structured
    //    walls (every marker on an integer x plane, and at each (y, z) position one marker on every
    //    x plane: the rings of a straight pipe) keep each line together, so that marker
    //    line * nx + x is the line's marker on plane x.
    const int nx = n[0];
    std::vector<int64_t> line_key((size_t)M, 0);  // first original index of the marker's line
    bool lines = M > 0 && M % nx == 0;
    for (int64_t j = 0; j < M && lines; ++j) lines = xyz[j] == std::floor(xyz[j]);
    if (lines) {
        std::vector<int64_t> o((size_t)M);
        for (int64_t j = 0; j < M; ++j) o[j] = j;
        std::stable_sort(o.begin(), o.end(), [&](int64_t a, int64_t b) {
            if (xyz[M + a] != xyz[M + b]) return xyz[M + a] < xyz[M + b];
            if (xyz[2 * M + a] != xyz[2 * M + b]) return xyz[2 * M + a] < xyz[2 * M + b];
            return xyz[a] < xyz[b];
        });
        for (int64_t g0 = 0; g0 < M && lines; g0 += nx) {
            int64_t first = o[g0];
            for (int x = 0; x < nx && lines; ++x) {
                const int64_t j = o[g0 + x];
                lines = xyz[j] == (double)x && xyz[M + j] == xyz[M + o[g0]] && xyz[2 * M + j] == xyz[2 * M + o[g0]];
                first = std::min(first, j);
            }
            for (int x = 0; x < nx; ++x) line_key[o[g0 + x]] = first;
        }
    }
    std::vector<int64_t> perm((size_t)M);
    for (int64_t j = 0; j < M; ++j) perm[j] = j;
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) {
        const int ka = tcell[tptr[a]], kb = tcell[tptr[b]];
        const int ya = ka / nx, yb = kb / nx;
        if (ya != yb) return ya < yb;
        if (lines && line_key[a] != line_key[b]) return line_key[a] < line_key[b];
        return (ka % nx) < (kb % nx);
    });
    int tm = 1;
    for (int64_t j = 0; j < M; ++j) tm = std::max(tm, tptr[j + 1] - tptr[j]);
    std::vector<int> tap_cell((size_t)tm * M);
    std::vector<float> tap_w((size_t)tm * M, 0.f);
    std::vector<double> d((size_t)M);
    for (int64_t i = 0; i < M; ++i) {
        const int64_t j = perm[i];
        d[i] = d0[j];
        for (int t = 0; t < tm; ++t) {
            const int src = tptr[j] + t;
            const bool real = src < tptr[j + 1];
            tap_cell[(size_t)t * M + i] = real ? tcell[src] : tcell[tptr[j]];
            tap_w[(size_t)t * M + i] = real ? (float)tw[src] : 0.f;
        }
    }
    // 4. band cells in increasing index, each with its (internal marker, weight) entries in
    //    internal marker order: the taps listed marker by marker, stably sorted by cell
    struct Entry {
        int cell, mk;
        double w;
    };
    std::vector<Entry> ent;
    ent.reserve(T);
    for (int64_t i = 0; i < M; ++i) {
        const int64_t j = perm[i];
        for (int t = tptr[j]; t < tptr[j + 1]; ++t) ent.push_back({tcell[t], (int)i, tw[t]});
    }
    std::stable_sort(ent.begin(), ent.end(), [](const Entry &a, const Entry &b) { return a.cell < b.cell; });
    std::vector<size_t> start;  // first entry of each band cell
    for (size_t k = 0; k < ent.size(); ++k)
        if (k == 0 || ent[k].cell != ent[k - 1].cell) start.push_back(k);
    const int64_t nband = (int64_t)start.size();
    start.push_back(ent.size());
    int km = 1;
    for (int64_t e = 0; e < nband; ++e) km = std::max<int>(km, (int)(start[e + 1] - start[e]));
    if (nband * km > kBandSlots * s->Mcap)
        return fail(MHD_ERR_INVALID_ARG, "markers too dense: %lld wall cells x %d entries exceed the workspace",
                    (long long)nband, km);
    std::vector<int> band_cell((size_t)nband), band_mk((size_t)nband * km);
    std::vector<float> band_w((size_t)nband * km, 0.f);
    for (int64_t e = 0; e < nband; ++e) {
        const size_t a = start[e], cnt = start[e + 1] - a;
        band_cell[e] = ent[a].cell;
        for (int q = 0; q < km; ++q) {
            const bool real = q < (int)cnt;
            band_mk[(size_t)q * nband + e] = real ? ent[a + q].mk : ent[a].mk;
            band_w[(size_t)q * nband + e] = real ? (float)ent[a + q].w : 0.f;
        }
    }
    // 4b. line tables (n_x a multiple of 64, so a wave's 64 markers or band cells share one line
    //     or band row): the taps of line l are those of its marker on plane 0, shifted by x; the
    //     entries of band row r those of its cell on plane 0, with the line of each entry. Every
    //     marker and band cell is checked against the general tables, so the two forms read the
    //     same taps and entries in the same order.
    const int64_t nlines = lines ? M / nx : 0;
    const int64_t nrows = lines ? nband / nx : 0;
    bool ring = lines && nx % 64 == 0 && nband % nx == 0;
    std::vector<int> ring_tap, row_off, row_mk;
    std::vector<float> ring_tw, row_w;
    if (ring) {
        ring_tap.resize((size_t)(nlines * tm));
        ring_tw.resize((size_t)(nlines * tm));
        for (int64_t l = 0; l < nlines; ++l)
            for (int t = 0; t < tm; ++t) {
                ring_tap[(size_t)(l * tm + t)] = tap_cell[(size_t)t * M + l * nx];
                ring_tw[(size_t)(l * tm + t)] = tap_w[(size_t)t * M + l * nx];
            }
        for (int64_t i = 0; i < M && ring; ++i) {
            const int64_t l = i / nx, x = i % nx;
            for (int t = 0; t < tm && ring; ++t)
                ring = tap_cell[(size_t)t * M + i] == x + ring_tap[(size_t)(l * tm + t)] &&
                       tap_w[(size_t)t * M + i] == ring_tw[(size_t)(l * tm + t)];
        }
    }
    if (ring) {
        row_off.resize((size_t)nrows);
        row_mk.resize((size_t)(nrows * km));
        row_w.resize((size_t)(nrows * km));
        for (int64_t r = 0; r < nrows; ++r) {
            row_off[r] = band_cell[(size_t)(r * nx)];
            for (int q = 0; q < km; ++q) {
                row_mk[(size_t)(r * km + q)] = band_mk[(size_t)q * nband + r * nx] / nx;
                row_w[(size_t)(r * km + q)] = band_w[(size_t)q * nband + r * nx];
            }
        }
        for (int64_t e = 0; e < nband && ring; ++e) {
            const int64_t r = e / nx, x = e % nx;
            ring = band_cell[e] == x + row_off[r];
            for (int q = 0; q < km && ring; ++q)
                ring = band_mk[(size_t)q * nband + e] == row_mk[(size_t)(r * km + q)] * nx + x &&
                       band_w[(size_t)q * nband + e] == row_w[(size_t)(r * km + q)];
        }
        ring = ring && nlines * tm <= s->Mcap && nrows <= s->Mcap && nrows * km <= s->Mcap;
    }
    // 5. wall values in internal order
    std::vector<float> uw((size_t)(3 * M), 0.f), bw((size_t)(3 * M), 0.f);
    for (int64_t i = 0; i < M; ++i)
        for (int a = 0; a < 3; ++a) {
            if (u_wall) uw[(size_t)a * M + i] = (float)u_wall[a * M + perm[i]];
            if (b_wall) bw[(size_t)a * M + i] = (float)b_wall[a * M + perm[i]];
        }
    auto up = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(s->ws + off, src, bytes, hipMemcpyHostToDevice, s->stream);
    };
    // MHD_IB_RING: 0 = general tables only, 1 (default) = line tables where the wall allows,
    // 2 = line tables required (the call fails otherwise)
    const int ring_mode = env_int("MHD_IB_RING", 1);
    if (ring_mode == 2 && !ring)
        return fail(MHD_ERR_UNSUPPORTED, "MHD_IB_RING=2: the markers are not line-structured with n_x %% 64 == 0");
    HIPCHK(hipStreamSynchronize(s->stream));
    HIPCHK(up(s->L.tap_cell, tap_cell.data(), tap_cell.size() * sizeof(int)));
    HIPCHK(up(s->L.tap_w, tap_w.data(), tap_w.size() * sizeof(float)));
    HIPCHK(up(s->L.uwall, uw.data(), uw.size() * sizeof(float)));
    HIPCHK(up(s->L.bwall, bw.data(), bw.size() * sizeof(float)));
    HIPCHK(up(s->L.band_cell, band_cell.data(), band_cell.size() * sizeof(int)));
    HIPCHK(up(s->L.band_mk, band_mk.data(), band_mk.size() * sizeof(int)));
    HIPCHK(up(s->L.band_w, band_w.data(), band_w.size() * sizeof(float)));
    if (ring) {
        HIPCHK(up(s->L.ring_tap, ring_tap.data(), ring_tap.size() * sizeof(int)));
        HIPCHK(up(s->L.ring_tw, ring_tw.data(), ring_tw.size() * sizeof(float)));
        HIPCHK(up(s->L.row_off, row_off.data(), row_off.size() * sizeof(int)));
        HIPCHK(up(s->L.row_mk, row_mk.data(), row_mk.size() * sizeof(int)));
        HIPCHK(up(s->L.row_w, row_w.data(), row_w.size() * sizeof(float)));
    }
    HIPCHK(hipStreamSynchronize(s->stream));
    s->lines = ring;
    s->ring_on = ring && ring_mode != 0;
    s->M = M;
    s->nband = nband;
    s->tm = tm;
    s->km = km;
    s->d = std::move(d);
    if (s->owner) batch_touch(s->owner);
    mhd_status st = upload_scalings(s);
    if (st != MHD_OK) {  // the wall is dropped rather than left half-configured
        s->M = 0;
        s->nband = 0;
        return st;
    }
    return MHD_OK;
}

mhd_status mhd_set_params(mhd_sim *s, const mhd_params *p) {
    g_err.clear();
    if (!s || !p) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (!(p->nu > 0.0)) return fail(MHD_ERR_INVALID_ARG, "nu = %g must be > 0", p->nu);
    if (!std::isfinite(p->gamma)) return fail(MHD_ERR_INVALID_ARG, "non-finite gamma");
    if (fluid_branch_mac(*p) && gamma_of(*p) != 1.0)
        return fail(MHD_ERR_UNSUPPORTED, "tau = 3 nu / gamma + 1/2 = %g >= 1: the macroscopic branch has no rescaling (gamma = %g)",
                    3.0 * p->nu / gamma_of(*p) + 0.5, gamma_of(*p));
    if (!(p->eta > 0.0)) return fail(MHD_ERR_INVALID_ARG, "eta must be > 0");
    if (p->n_mag < 1) return fail(MHD_ERR_INVALID_ARG, "n_mag must be >= 1");
    if (p->bext_kind < 0 || p->bext_kind > 3) return fail(MHD_ERR_INVALID_ARG, "unknown bext_kind %d", p->bext_kind);
    if (p->bext_kind == MHD_BEXT_SIX_MAGNETS && !(p->avg_radius > 0.0))
        return fail(MHD_ERR_INVALID_ARG, "the six-magnet field needs avg_radius > 0");
    if (p->bext_kind == MHD_BEXT_TANH_FRINGE_Y && !(p->fringe_w > 0.0))
        return fail(MHD_ERR_INVALID_ARG, "fringe_w must be > 0");
    if (p->flow_control && !(p->avg_radius > 0.0)) return fail(MHD_ERR_INVALID_ARG, "flow control needs avg_radius > 0");
    if (p->lattice != 0 && p->lattice != 19 && p->lattice != 27)
        return fail(MHD_ERR_INVALID_ARG, "lattice %d: use 19 (D3Q19, also 0) or 27 (D3Q27)", p->lattice);
    const double alpha_min = p->lattice == 27 ? 13.0 / 27.0 : 4.0 / 9.0;
    if (p->alpha != 0.0 && !(p->alpha >= alpha_min))
        return fail(MHD_ERR_INVALID_ARG, "alpha = %g: the accelerated sweep needs alpha >= %g on this lattice (or 0)",
                    p->alpha, alpha_min);
    if (p->lattice == 27 && !(s->g.rho_storage == MHD_STORE_F32 && s->g.u_storage == MHD_STORE_F32))
        return fail(MHD_ERR_UNSUPPORTED, "D3Q27 is built for float32 and split storage only");
    for (double v : {p->nu, p->eta, p->lambda_u, p->lambda_b, p->G0, p->G1, p->period, p->B0, p->fringe_x0, p->fringe_w,
                     p->yc, p->zc, p->avg_radius, p->u_bulk_target, p->k_c, p->alpha, p->magnet_half_width,
                     p->magnet_distance, p->omega_radius})
        if (!std::isfinite(v)) return fail(MHD_ERR_INVALID_ARG, "non-finite parameter");
    const bool first = !s->have_params;
    const mhd_params old = s->prm;
    drop_step_graphs(s);
    s->fused_lf = env_int("MHD_FUSED_LF", 1) != 0;
    s->prm = *p;
    s->have_params = true;
    if (s->owner) batch_touch(s->owner);
    mhd_status st = upload_scalings(s);
    if (st != MHD_OK) {
        s->prm = old;
        s->have_params = !first;
        return st;
    }
    STEPCHK(upload_bext(s));
    // cells of the flow-rate region r <= R
    int64_t cnt = 0;
    const double R2 = p->avg_radius * p->avg_radius;
    for (int z = 0; z < s->g.nz; ++z)
        for (int y = 0; y < s->g.ny; ++y) {
            const double dy = y - p->yc, dz = z - p->zc;
            if (dy * dy + dz * dz <= R2) cnt += s->g.nx;
        }
    s->flow_inv_count = cnt ? 1.0 / (double)cnt : 0.0;
    if (first) {  // the controlled force starts from G0
        DevCtrl h;
        STEPCHK(read_ctrl(s, &h));
        h.G = p->G0;
        HIPCHK(hipMemcpyAsync(s->ctrl(), &h, sizeof h, hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return MHD_OK;
}

mhd_status mhd_set_field(mhd_sim *s, mhd_field f, const double *host) {
    g_err.clear();
    if (!s || !host) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (f < MHD_FIELD_RHO || f > MHD_FIELD_B_INDUCED) return fail(MHD_ERR_INVALID_ARG, "unknown field %d", (int)f);
    const int64_t n = (f == MHD_FIELD_RHO ? 1 : 3) * s->N;
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return fail(MHD_ERR_INVALID_ARG, "non-finite value at index %lld", (long long)i);
    HIPCHK(hipStreamSynchronize(s->stream));
    return fill_field(s, f, host, false);
}

mhd_status mhd_get_field(mhd_sim *s, mhd_field f, double *host) {
    g_err.clear();
    if (!s || !host) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (f < MHD_FIELD_RHO || f > MHD_FIELD_B_INDUCED) return fail(MHD_ERR_INVALID_ARG, "unknown field %d", (int)f);
    const int ncomp = f == MHD_FIELD_RHO ? 1 : 3;
    const int64_t n = ncomp * s->N;
    int kind;
    double scale = 1.0, offset = 0.0;
    const void *src;
    if (f == MHD_FIELD_RHO) {
        kind = s->g.rho_storage;
        offset = 1.0;
        src = s->rho(s->cr);
    } else if (f == MHD_FIELD_U) {
        kind = s->g.u_storage;
        if (kind != MHD_STORE_F32) scale = s->g.u_scale;
        src = s->u(s->cu);
    } else {
        kind = s->g.b_storage;
        if (kind != MHD_STORE_F32) scale = s->g.b_scale;
        src = s->b(s->cb);
    }
    float *stage = s->at<float>(s->L.F);
    HIPCHK(launch_load_kind(s->stream, kind, src, stage, n));
    std::vector<float> tmp((size_t)n);
    HIPCHK(hipMemcpyAsync(tmp.data(), stage, n * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int64_t i = 0; i < n; ++i) host[i] = (double)tmp[i] * scale + offset;
    if (f == MHD_FIELD_B_INDUCED && s->split()) {  // b = (hi + lo) b_scale
        HIPCHK(launch_load_kind(s->stream, MHD_STORE_F16, s->bh(s->ch), stage, n));
        HIPCHK(hipMemcpyAsync(tmp.data(), stage, n * sizeof(float), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        for (int64_t i = 0; i < n; ++i) host[i] += (double)tmp[i] * scale;
    }
    DevCtrl h;
    STEPCHK(read_ctrl(s, &h));
    if (h.status & 1) return fail(MHD_ERR_UNSTABLE, "a fluid step or a budget pass found non-finite values or |u| >= c_s");
    return MHD_OK;
}

mhd_status mhd_get_time(mhd_sim *s, int64_t *t, double *G) {
    g_err.clear();
    if (!s) return fail(MHD_ERR_INVALID_ARG, "sim is NULL");
    DevCtrl h;
    STEPCHK(read_ctrl(s, &h));
    if (t) *t = h.t;
    if (G) *G = h.G;
    return MHD_OK;
}

mhd_status mhd_set_time(mhd_sim *s, int64_t t, double G) {
    g_err.clear();
    if (!s) return fail(MHD_ERR_INVALID_ARG, "sim is NULL");
    if (t < 0 || !std::isfinite(G)) return fail(MHD_ERR_INVALID_ARG, "t must be >= 0 and G finite");
    DevCtrl h;
    STEPCHK(read_ctrl(s, &h));
    h.t = t;
    h.G = G;
    h.G_step = G;
    HIPCHK(hipMemcpyAsync(s->ctrl(), &h, sizeof h, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->t_host = t;
    return MHD_OK;
}

mhd_status mhd_step(mhd_sim *s, int64_t n_steps, int32_t budget_every) {
    g_err.clear();
    STEPCHK(step_checks(s, n_steps));
    // On a caller stream the step is captured once per buffer state and replayed as a HIP graph
    // (one launch call per step instead of about 3 n_mag + 6); profiling steps launch directly.
    const bool graph = s->graph_on && s->stream != nullptr && !s->prof;
    for (int64_t i = 0; i < n_steps; ++i) {
        if (graph) {
            const int key = s->cb | (s->cr << 1) | (s->cu << 2) | (s->ch << 3);
            auto it = std::find_if(s->graphs.begin(), s->graphs.end(), [&](const mhd_sim::StepGraph &g) { return g.key == key; });
            if (it == s->graphs.end()) {
                const int cb = s->cb, cr = s->cr, cu = s->cu, ch = s->ch;
                const int64_t t = s->t_host;
                hipGraph_t g = nullptr;
                HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeRelaxed));
                const mhd_status st = one_step(s);
                const hipError_t ec = hipStreamEndCapture(s->stream, &g);
                mhd_sim::StepGraph sg{key, s->cb, s->cr, s->cu, s->ch, nullptr};
                s->cb = cb;  // the capture ran the host side of the step; the replay below runs it
                s->cr = cr;
                s->cu = cu;
                s->ch = ch;
                s->t_host = t;
                if (st != MHD_OK) {
                    if (ec == hipSuccess && g) (void)hipGraphDestroy(g);
                    return st;
                }
                if (ec != hipSuccess) return fail(MHD_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
                const hipError_t ei = hipGraphInstantiate(&sg.exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ei != hipSuccess) return fail(MHD_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
                s->graphs.push_back(sg);
                it = s->graphs.end() - 1;
            }
            HIPCHK(hipGraphLaunch(it->exec, s->stream));
            s->cb = it->cb;
            s->cr = it->cr;
            s->cu = it->cu;
            s->ch = it->ch;
            s->t_host += 1;
        } else {
            STEPCHK(one_step(s));
        }
        if (budget_every > 0 && s->t_host % budget_every == 0) STEPCHK(record_budget(s));
    }
    return MHD_OK;
}

}  // extern "C"

namespace mhd {

mhd_status report_error(mhd_status st, const char *msg) { return fail(st, "%s", msg); }

// Step scratch regions of a box, each 256-byte aligned: F [3][N] float32, wall corrections
// [3][M] float32, flow partials [kRedBlocks] and budget partials [kRedBlocks][kBudgetVals] float64.
static size_t scratch_layout(const mhd_sim *s, size_t off[4]) {
    const size_t sizes[4] = {3 * (size_t)s->N * sizeof(float), 3 * (size_t)std::max<int64_t>(s->Mcap, 1) * sizeof(float),
                             (size_t)kRedBlocks * sizeof(double), (size_t)kRedBlocks * kBudgetVals * sizeof(double)};
    size_t o = 0;
    for (int i = 0; i < 4; ++i) {
        off[i] = o;
        o = align256(o + sizes[i]);
    }
    return o;
}

size_t step_scratch_bytes(const mhd_sim *s) {
    size_t off[4];
    return scratch_layout(s, off);
}

mhd_status step_in_scratch(mhd_sim *s, int64_t n_steps, int32_t budget_every, void *dev_scratch) {
    size_t off[4];
    scratch_layout(s, off);
    char *base = static_cast<char *>(dev_scratch);
    s->scr.F = reinterpret_cast<float *>(base + off[0]);
    s->scr.delta = reinterpret_cast<float *>(base + off[1]);
    s->scr.flow = reinterpret_cast<double *>(base + off[2]);
    s->scr.red = reinterpret_cast<double *>(base + off[3]);
    mhd_status st = MHD_OK;
    for (int64_t i = 0; i < n_steps && st == MHD_OK; ++i) {  // direct launches: no graph holds these pointers
        st = one_step(s);
        if (st == MHD_OK && budget_every > 0 && s->t_host % budget_every == 0) st = record_budget(s);
    }
    s->scr = mhd_sim::Scratch{};
    return st;
}

mhd_status step_checks(mhd_sim *s, int64_t n_steps) {
    if (!s) return fail(MHD_ERR_INVALID_ARG, "sim is NULL");
    if (s->owner) return fail(MHD_ERR_STATE, "this box belongs to a batch: step it with mhd_batch_step");
    if (!s->have_params) return fail(MHD_ERR_STATE, "mhd_set_params must be called before stepping");
    if (n_steps < 0) return fail(MHD_ERR_INVALID_ARG, "n_steps < 0");
    return MHD_OK;
}

int sim_device(const mhd_sim *s) { return s->device; }

}  // namespace mhd

extern "C" {

mhd_status mhd_set_graph(mhd_sim *s, int32_t enable) {
    g_err.clear();
    if (!s) return fail(MHD_ERR_INVALID_ARG, "sim is NULL");
    if (enable != 0 && enable != 1) return fail(MHD_ERR_INVALID_ARG, "enable must be 0 or 1");
    s->graph_on = enable != 0;
    if (!s->graph_on) drop_step_graphs(s);
    return MHD_OK;
}

mhd_status mhd_tune(mhd_sim *s, int32_t reps) {
    g_err.clear();
    if (!s) return fail(MHD_ERR_INVALID_ARG, "sim is NULL");
    if (s->owner) return fail(MHD_ERR_STATE, "this box belongs to a batch: tune it with mhd_batch_tune");
    if (!s->have_params) return fail(MHD_ERR_STATE, "mhd_set_params must be called before mhd_tune");
    if (reps <= 0) reps = 5;
    const StepConst c = step_const(s);
    const int nx = s->g.nx, nz = s->g.nz;
    std::vector<SweepLaunch> cand;
    for (int zc : {4, 8, 16, 32, 64, 128}) {
        if (zc > 2 * nz && zc != 4) continue;
        if (nx % 128 == 0)
            for (int ty : {4, 8}) cand.push_back({64, ty, zc, 1});
        for (int tx : {64, 32, 16, 8})
            if (tx <= std::max(8, nx)) cand.push_back({tx, 4, zc, 0});
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(MHD_ERR_HIP, "hipEventCreate failed");
    }
    // Each candidate runs reps sweeps of the live state into the other buffer of b, which the
    // next step overwrites (the split form's hi part is only read): the state is unchanged.
    SweepLaunch best_L = s->sweep;
    float best = 0.f;
    mhd_status st = MHD_OK;
    for (size_t i = 0; i < cand.size() && st == MHD_OK; ++i) {
        const SweepLaunch L = cand[i];
        SweepArgs a = make_sweep_args(s->split() ? s->u16() : s->u(s->cu), s->b(s->cb), s->b(1 - s->cb),
                                      s->at<float>(s->L.bext), c, L);
        a.bext_yz = s->byz();
        if (s->split()) {
            a.u_scale = c.copy_scale;
            a.bh = s->bh(s->ch);
        }
        hipError_t e = launch_mag_sweep(s->stream, s->kinds, a, L);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_mag_sweep(s->stream, s->kinds, a, L);
        if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = fail(MHD_ERR_HIP, "timing a sweep failed: %s", hipGetErrorString(e));
            break;
        }
        if (i == 0 || ms < best) {
            best = ms;
            best_L = L;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != MHD_OK) return st;
    s->sweep.tx = best_L.tx;
    s->sweep.ty = best_L.ty;
    s->sweep.zchunk = best_L.zchunk;
    s->sweep.pair = best_L.pair;
    drop_step_graphs(s);
    return MHD_OK;
}

mhd_status mhd_mag_residual_curve(mhd_sim *s, int32_t n_sweeps, double *res_out) {
    g_err.clear();
    if (!s || !res_out) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (!s->have_params) return fail(MHD_ERR_STATE, "mhd_set_params must be called first");
    if (n_sweeps < 1 || n_sweeps > kResCap) return fail(MHD_ERR_INVALID_ARG, "n_sweeps must be in [1, %d]", kResCap);
    const StepConst c = step_const(s);
    hipStream_t st = s->stream;
    // save b (float32, or the split form's lo and hi: 12 N bytes either way) in the staging area
    char *stage = reinterpret_cast<char *>(s->at<float>(s->L.F));
    const size_t bbytes = 3 * (size_t)s->N * kind_bytes(s->g.b_storage);
    const int cb0 = s->cb, ch0 = s->ch;
    HIPCHK(hipMemcpyAsync(stage, s->b(cb0), bbytes, hipMemcpyDeviceToDevice, st));
    if (s->split()) HIPCHK(hipMemcpyAsync(stage + bbytes, s->bh(ch0), 3 * (size_t)s->N * 2, hipMemcpyDeviceToDevice, st));
    double *res = s->at<double>(s->L.res);
    mhd_status result = MHD_OK;
    for (int k = 0; k < n_sweeps && result == MHD_OK; ++k) {
        result = mag_iteration(s, c, k);
        if (result != MHD_OK) break;
        hipError_t e = launch_budget(st, s->kinds, s->rho(s->cr), s->u(s->cu), s->b(s->cb), s->bh(s->ch),
                                     s->at<float>(s->L.bext), s->byz(), s->ctrl(), s->at<double>(s->L.red_part),
                                     nullptr, c);
        if (e == hipSuccess) e = launch_residual_final(st, s->at<double>(s->L.red_part), res + k);
        if (e != hipSuccess) result = fail(MHD_ERR_HIP, "residual pass failed: %s", hipGetErrorString(e));
    }
    // restore the induced field and its buffer state
    s->cb = cb0;
    s->ch = ch0;
    HIPCHK(hipMemcpyAsync(s->b(cb0), stage, bbytes, hipMemcpyDeviceToDevice, st));
    if (s->split()) HIPCHK(hipMemcpyAsync(s->bh(ch0), stage + bbytes, 3 * (size_t)s->N * 2, hipMemcpyDeviceToDevice, st));
    if (result != MHD_OK) {
        (void)hipStreamSynchronize(st);
        return result;
    }
    HIPCHK(hipMemcpyAsync(res_out, res, (size_t)n_sweeps * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return MHD_OK;
}

mhd_status mhd_choose_n_mag(mhd_sim *s, double tol, int32_t n_max, int32_t apply, int32_t *n_out) {
    g_err.clear();
    if (!s || !n_out) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (!(tol > 0.0 && tol < 1.0)) return fail(MHD_ERR_INVALID_ARG, "tol = %g must lie in (0, 1)", tol);
    if (apply != 0 && apply != 1) return fail(MHD_ERR_INVALID_ARG, "apply must be 0 or 1");
    std::vector<double> res((size_t)std::max(n_max, 1));
    STEPCHK(mhd_mag_residual_curve(s, n_max, res.data()));
    int32_t n = n_max;
    for (int32_t k = 0; k < n_max; ++k)
        if (res[(size_t)k] <= tol * res[0]) {
            n = k + 1;
            break;
        }
    if (apply) {
        mhd_params p = s->prm;
        p.n_mag = n;
        STEPCHK(mhd_set_params(s, &p));
    }
    *n_out = n;
    return MHD_OK;
}

mhd_status mhd_record_budget(mhd_sim *s) {
    g_err.clear();
    if (!s) return fail(MHD_ERR_INVALID_ARG, "sim is NULL");
    if (!s->have_params) return fail(MHD_ERR_STATE, "mhd_set_params must be called first");
    return record_budget(s);
}

mhd_status mhd_get_budgets(mhd_sim *s, mhd_budget *out, int64_t cap, int64_t *n_out) {
    g_err.clear();
    if (!s || !n_out) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (cap > 0 && !out) return fail(MHD_ERR_INVALID_ARG, "out is NULL");
    DevCtrl h;
    STEPCHK(read_ctrl(s, &h));
    const int64_t n = std::min<int64_t>(h.n_records, std::max<int64_t>(cap, 0));
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(out, s->at<mhd_budget>(s->L.ring), n * sizeof(mhd_budget), hipMemcpyDeviceToHost,
                              s->stream));
    }
    HIPCHK(launch_reset_records(s->stream, s->ctrl()));
    HIPCHK(hipStreamSynchronize(s->stream));
    *n_out = n;
    if (h.status & 1) return fail(MHD_ERR_UNSTABLE, "a fluid step or a budget pass found non-finite values or |u| >= c_s");
    return MHD_OK;
}

mhd_status mhd_set_profiling(mhd_sim *s, int32_t enable) {
    g_err.clear();
    if (!s) return fail(MHD_ERR_INVALID_ARG, "sim is NULL");
    s->prof = enable != 0;
    return MHD_OK;
}

mhd_status mhd_kernel_stats(mhd_sim *s, int32_t kernel, int64_t *launches, double *total_ms) {
    g_err.clear();
    if (!s || !launches || !total_ms) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (kernel < 0 || kernel >= MHD_K_COUNT) return fail(MHD_ERR_INVALID_ARG, "unknown kernel id %d", kernel);
    HIPCHK(hipStreamSynchronize(s->stream));
    double tot = 0.0;
    for (size_t i = 0; i < s->ev_used[kernel]; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, s->ev_pool[kernel][i].a, s->ev_pool[kernel][i].b));
        tot += ms;
    }
    *launches = (int64_t)s->ev_used[kernel];
    *total_ms = tot;
    s->ev_used[kernel] = 0;
    return MHD_OK;
}

mhd_status mhd_destroy(mhd_sim *s) {
    g_err.clear();
    if (!s) return MHD_OK;
    if (s->owner) return fail(MHD_ERR_STATE, "this box belongs to a batch: free it with mhd_batch_destroy");
    drop_step_graphs(s);
    (void)hipStreamSynchronize(s->stream);
    for (int k = 0; k < MHD_K_COUNT; ++k)
        for (auto &e : s->ev_pool[k]) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
    delete s;
    return MHD_OK;
}

}  // extern "C"

// =============================================================================================
// Batched form: many boxes advanced by shared launches (see the kernels' PipeStep / BlockMap)
// =============================================================================================
namespace {

// Upper bound of the workgroups of one box in any batched launch kind.
int64_t sweep_blocks_bound(const mhd_grid_desc &g) {
    int64_t m = 0;
    for (int tx : {64, 32, 16, 8}) {
        const int ty = 256 / tx;
        m = std::max<int64_t>(m, (int64_t)((g.nx + tx - 1) / tx) * ((g.ny + ty - 1) / ty) * g.nz);
    }
    return m;
}
int64_t blocks_of(int64_t n, int t) { return (n + t - 1) / t; }
int64_t map_bound(const mhd_pipe_desc &p) {
    const int64_t N = (int64_t)p.grid.nx * p.grid.ny * p.grid.nz;
    return sweep_blocks_bound(p.grid) + blocks_of(p.n_markers, kIbThreads) + blocks_of(27 * p.n_markers, kIbThreads) +
           blocks_of(N, kCellThreads);
}

struct BatchLayout {
    std::vector<size_t> pipe;  // workspace offset of every box
    std::vector<size_t> pipe_bytes;
    size_t tab[2] = {0, 0};    // PipeStep[n] of the two buffer phases
    size_t map = 0;            // BlockMap[map_cap]
    int64_t map_cap = 0;
    size_t total = 0;
};

BatchLayout make_batch_layout(const mhd_pipe_desc *p, int n) {
    BatchLayout L;
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        const size_t sz = make_layout(p[i].grid, p[i].n_markers).total;
        L.pipe.push_back(off);
        L.pipe_bytes.push_back(sz);
        off = align256(off + sz);
        L.map_cap += map_bound(p[i]);
    }
    for (int k = 0; k < 2; ++k) {
        L.tab[k] = off;
        off = align256(off + (size_t)n * sizeof(PipeStep));
    }
    L.map = off;
    off = align256(off + (size_t)L.map_cap * sizeof(BlockMap));
    L.total = off;
    return L;
}

mhd_status check_pipes(const mhd_pipe_desc *p, int32_t n) {
    if (!p) return fail(MHD_ERR_INVALID_ARG, "pipe descriptors are NULL");
    if (n < 1 || n > (1 << 16)) return fail(MHD_ERR_INVALID_ARG, "n = %d pipes outside [1, 65536]", n);
    for (int i = 0; i < n; ++i) {
        STEPCHK(check_desc(&p[i].grid));
        if (p[i].n_markers < 0 || p[i].n_markers >= ((int64_t)1 << 26))
            return fail(MHD_ERR_INVALID_ARG, "pipe %d: n_markers must be in [0, 2^26)", i);
        const mhd_grid_desc &a = p[0].grid, &b = p[i].grid;
        if (a.rho_storage != b.rho_storage || a.u_storage != b.u_storage || a.b_storage != b.b_storage)
            return fail(MHD_ERR_UNSUPPORTED, "pipe %d: all pipes of a batch must share the storage kinds", i);
    }
    return MHD_OK;
}

struct BatchSlot {  // launch tables (and graph) of one state of the boxes' double buffers
    bool valid = false;
    int64_t version = -1;
    std::vector<int> sig;
    hipGraphExec_t exec = nullptr;
};

struct BatchGroup {  // boxes sharing one sweep kernel (tile form), largest n_mag first
    SweepLaunch L{};
    int64_t map_base = 0;
    std::vector<int> pipes;
    std::vector<int> nmag;
    std::vector<int64_t> cum;  // cum[i] = workgroups of the first i boxes
};

}  // namespace

struct mhd_batch {
    int n = 0;
    std::vector<mhd_sim *> pipes;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    BatchLayout L;
    int kinds = 0, kind_u = 0, kind_b = 0;
    bool graph = true, prof = false;
    // launch plan, rebuilt whenever parameters, markers or tiles of a box change
    int64_t version = 0, plan_version = -1;
    std::vector<int> order;   // boxes by n_mag, largest first
    std::vector<int> nmag;    // n_mag of order[i]
    int max_nmag = 0;
    std::vector<BatchGroup> groups;
    int64_t interp_base = 0, spread_base = 0, cell_base = 0;
    std::vector<int64_t> cum_interp, cum_spread, cum_cells;  // over `order`
    bool any_flow = false;
    bool q27 = false;  // lattice of the batch (one for all pipes)
    BatchSlot slot[2];
    int next_slot = 0;
    std::vector<Event2> ev_pool[MHD_K_COUNT];
    size_t ev_used[MHD_K_COUNT] = {};

    PipeStep *tab(int k) const { return reinterpret_cast<PipeStep *>(ws + L.tab[k]); }
    BlockMap *map() const { return reinterpret_cast<BlockMap *>(ws + L.map); }
};

namespace {

void batch_touch(mhd_batch *b) { b->version += 1; }

// number of leading entries of a descending list that exceed r
int active_count(const std::vector<int> &desc, int r) {
    return (int)(std::upper_bound(desc.begin(), desc.end(), r, [](int v, int x) { return v > x; }) - desc.begin());
}

void drop_graphs(mhd_batch *b) {
    for (auto &sl : b->slot) {
        if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
        sl.exec = nullptr;
        sl.valid = false;
    }
}

mhd_status build_plan(mhd_batch *b) {
    for (int i = 0; i < b->n; ++i)
        if (!b->pipes[i]->have_params) return fail(MHD_ERR_STATE, "pipe %d has no parameters (mhd_set_params)", i);
    HIPCHK(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    b->order.resize(b->n);
    for (int i = 0; i < b->n; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return b->pipes[x]->prm.n_mag > b->pipes[y]->prm.n_mag; });
    b->nmag.resize(b->n);
    for (int i = 0; i < b->n; ++i) b->nmag[i] = b->pipes[b->order[i]]->prm.n_mag;
    b->max_nmag = b->nmag[0];
    std::vector<BlockMap> map;
    // sweep groups, one per tile form
    b->groups.clear();
    for (auto *s : b->pipes)
        if ((s->prm.lattice == 27) != (b->pipes[0]->prm.lattice == 27))
            return fail(MHD_ERR_UNSUPPORTED, "all pipes of a batch must use the same lattice");
    b->q27 = b->pipes[0]->prm.lattice == 27;
    auto key = [](const SweepLaunch &L) { return (L.pair ? 100 + L.ty : L.tx) + 1000 * L.byz; };
    for (int p : b->order) {
        mhd_sim *s = b->pipes[p];
        SweepLaunch e = effective_tiles(s->sweep, s->g.nx);
        e.byz = s->byz() != nullptr;
        e.q27 = b->q27;
        BatchGroup *g = nullptr;
        for (auto &x : b->groups)
            if (key(x.L) == key(e)) g = &x;
        if (!g) {
            b->groups.emplace_back();
            g = &b->groups.back();
            g->L = e;
        }
        g->pipes.push_back(p);
        g->nmag.push_back(s->prm.n_mag);
    }
    for (auto &g : b->groups) {
        g.map_base = (int64_t)map.size();
        g.cum.assign(1, 0);
        for (int p : g.pipes) {
            mhd_sim *s = b->pipes[p];
            const SweepArgs a = make_sweep_args(nullptr, nullptr, nullptr, nullptr, step_const(s),
                                                effective_tiles(s->sweep, s->g.nx));
            for (int lb = 0; lb < a.nblocks; ++lb) map.push_back({p, lb});
            g.cum.push_back(g.cum.back() + a.nblocks);
        }
    }
    auto add_list = [&](int64_t &base, std::vector<int64_t> &cum, auto count) {
        base = (int64_t)map.size();
        cum.assign(1, 0);
        for (int p : b->order) {
            const int64_t nb = blocks_of(count(b->pipes[p]), kIbThreads);
            for (int64_t lb = 0; lb < nb; ++lb) map.push_back({p, (int)lb});
            cum.push_back(cum.back() + nb);
        }
    };
    add_list(b->interp_base, b->cum_interp, [](mhd_sim *s) { return s->M; });
    add_list(b->spread_base, b->cum_spread, [](mhd_sim *s) { return s->M ? s->nband : 0; });
    add_list(b->cell_base, b->cum_cells, [](mhd_sim *s) { return s->N; });
    if ((int64_t)map.size() > b->L.map_cap)
        return fail(MHD_ERR_OOM, "batch launch map needs %zu entries, %lld reserved", map.size(),
                    (long long)b->L.map_cap);
    for (int64_t v : b->cum_cells)
        if (v >= ((int64_t)1 << 31)) return fail(MHD_ERR_INVALID_ARG, "batch too large for one launch");
    b->any_flow = false;
    for (auto *s : b->pipes) b->any_flow = b->any_flow || s->prm.flow_control;
    HIPCHK(hipMemcpyAsync(b->map(), map.data(), map.size() * sizeof(BlockMap), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    b->plan_version = b->version;
    return MHD_OK;
}

IbArgs ib_args(mhd_sim *s, const float *sj, const float *wall) {
    IbArgs a;
    a.phi_hi = nullptr;
    a.copy = nullptr;
    a.copy_inv = 0.f;
    a.N = s->N;
    a.M = (int)s->M;
    a.nband = (int)s->nband;
    a.tm = s->tm;
    a.km = s->km;
    a.tap_cell = s->at<int>(s->L.tap_cell);
    a.tap_w = s->at<float>(s->L.tap_w);
    a.sj = sj;
    a.wall = wall;
    a.band_cell = s->at<int>(s->L.band_cell);
    a.band_mk = s->at<int>(s->L.band_mk);
    a.band_w = s->at<float>(s->L.band_w);
    a.delta = s->at<float>(s->L.delta);
    a.ring = s->ring_on ? 1 : 0;
    a.nx = s->g.nx;
    a.kmr = s->km;
    a.ring_tap = s->at<int>(s->L.ring_tap);
    a.ring_tw = s->at<float>(s->L.ring_tw);
    a.row_off = s->at<int>(s->L.row_off);
    a.row_mk = s->at<int>(s->L.row_mk);
    a.row_w = s->at<float>(s->L.row_w);
    return a;
}

// Launch arguments of one box for its current buffer state (one fluid step).
PipeStep pipe_step(mhd_sim *s) {
    PipeStep q{};
    const StepConst c = step_const(s);
    const SweepLaunch e = effective_tiles(s->sweep, s->g.nx);
    const float *bext = s->at<float>(s->L.bext);
    const int cb = s->cb, cu = s->cu, cr = s->cr, ch = s->ch;
    const void *us = s->split() ? s->u16() : s->u(cu);
    q.sw[0] = make_sweep_args(us, s->b(cb), s->b(1 - cb), bext, c, e);
    q.sw[1] = make_sweep_args(us, s->b(1 - cb), s->b(cb), bext, c, e);
    q.sw[0].bext_yz = q.sw[1].bext_yz = s->byz();
    q.sw[2] = q.sw[0];
    if (s->split()) {  // round 0 re-splits hi(ch) -> hi(1 - ch); later rounds read the new hi
        for (auto &w : q.sw) {
            w.u_scale = c.copy_scale;
            w.bh = s->bh(1 - ch);
        }
        q.sw[0].bh = s->bh(ch);
        q.sw[0].bho = s->bh(1 - ch);
    }
    IbArgs ab = ib_args(s, s->at<float>(s->L.s_b), s->at<float>(s->L.bwall));
    ab.phi_hi = s->bh(1 - ch);
    q.ib[0] = ab;
    q.ib[1] = ab;
    q.ib[2] = ib_args(s, s->at<float>(s->L.s_u), s->at<float>(s->L.uwall));
    q.ib[2].copy = s->u16();
    q.ib[2].copy_inv = c.inv_copy_scale;
    q.phi[0] = s->b(1 - cb);
    q.phi[1] = s->b(cb);
    q.phi[2] = s->u(1 - cu);
    q.scale[0] = q.scale[1] = c.b_scale;
    q.inv_scale[0] = q.inv_scale[1] = c.inv_b_scale;
    q.scale[2] = c.u_scale;
    q.inv_scale[2] = c.inv_u_scale;
    q.b_last = s->b((s->prm.n_mag & 1) ? 1 - cb : cb);
    q.b_hi = s->split() ? s->bh(1 - ch) : nullptr;
    q.bext_yz = s->byz();
    q.u_copy = s->u16();
    q.bext = bext;
    q.ctrl = s->ctrl();
    q.F = s->at<float>(s->L.F);
    q.rho = s->rho(cr);
    q.u = s->u(cu);
    q.rho_o = s->rho(1 - cr);
    q.u_o = s->u(1 - cu);
    q.flow_part = s->at<double>(s->L.flow_part);
    q.inv_count = s->flow_inv_count;
    q.c = c;
    return q;
}

std::vector<int> buffer_sig(const mhd_batch *b) {
    std::vector<int> v(b->n);
    for (int i = 0; i < b->n; ++i)
        v[i] = b->pipes[i]->cr | (b->pipes[i]->cu << 1) | (b->pipes[i]->cb << 2) | (b->pipes[i]->ch << 3);
    return v;
}

Event2 *next_event_b(mhd_batch *b, int k) {
    if (b->ev_used[k] == b->ev_pool[k].size()) {
        Event2 x;
        if (hipEventCreate(&x.a) != hipSuccess || hipEventCreate(&x.b) != hipSuccess) return nullptr;
        b->ev_pool[k].push_back(x);
    }
    return &b->ev_pool[k][b->ev_used[k]++];
}

template <typename Fn>
mhd_status timed_b(mhd_batch *b, int k, const char *what, Fn fn) {
    Event2 *e = nullptr;
    if (b->prof) {
        e = next_event_b(b, k);
        if (!e) return fail(MHD_ERR_HIP, "hipEventCreate failed");
        HIPCHK(hipEventRecord(e->a, b->stream));
    }
    hipError_t err = fn();
    if (err != hipSuccess) return fail(MHD_ERR_HIP, "batched launch of %s failed: %s", what, hipGetErrorString(err));
    if (e) HIPCHK(hipEventRecord(e->b, b->stream));
    return MHD_OK;
}

// The launch sequence of one fluid step of the whole batch, arguments from table slot k.
mhd_status issue_step(mhd_batch *b, int k) {
    hipStream_t st = b->stream;
    const PipeStep *tab = b->tab(k);
    const BlockMap *map = b->map();
    const int n = b->n;
    STEPCHK(timed_b(b, MHD_K_CONTROL, "ctrl_begin", [&] { return launch_ctrl_begin_batch(st, tab, n); }));
    for (int r = 0; r < b->max_nmag; ++r) {
        for (const auto &g : b->groups) {
            const int64_t nb = g.cum[active_count(g.nmag, r)];
            if (nb == 0) continue;
            Event2 *e = nullptr;
            if (b->prof && !(e = next_event_b(b, MHD_K_MAG_SWEEP))) return fail(MHD_ERR_HIP, "hipEventCreate failed");
            const int which = r == 0 ? 0 : (r & 1) ? 1 : 2;
            const hipError_t err = launch_mag_sweep_batch(st, b->kinds, g.L, tab, map + g.map_base, which, (int)nb,
                                                          e ? e->a : nullptr, e ? e->b : nullptr);
            if (err != hipSuccess) return fail(MHD_ERR_HIP, "batched launch of mag_sweep failed: %s", hipGetErrorString(err));
        }
        const int a = active_count(b->nmag, r);
        const int64_t ni = b->cum_interp[a], ns = b->cum_spread[a];
        if (ni > 0)
            STEPCHK(timed_b(b, MHD_K_IB, "wall correction", [&] {
                hipError_t e = launch_ib_interp_batch(st, b->kind_b, tab, map + b->interp_base, r & 1, (int)ni);
                if (e != hipSuccess) return e;
                return launch_ib_spread_batch(st, b->kind_b, tab, map + b->spread_base, r & 1, (int)ns);
            }));
    }
    const int nc = (int)b->cum_cells[n];
    STEPCHK(timed_b(b, MHD_K_LORENTZ, "lorentz",
                    [&] { return launch_lorentz_batch(st, b->kind_b, tab, map + b->cell_base, nc, b->q27); }));
    STEPCHK(timed_b(b, MHD_K_FLUID, "fluid",
                    [&] { return launch_fluid_batch(st, b->kinds, tab, map + b->cell_base, nc, b->q27); }));
    const int64_t ni = b->cum_interp[n], ns = b->cum_spread[n];
    if (ni > 0)
        STEPCHK(timed_b(b, MHD_K_IB, "wall correction", [&] {
            hipError_t e = launch_ib_interp_batch(st, b->kind_u, tab, map + b->interp_base, 2, (int)ni);
            if (e != hipSuccess) return e;
            return launch_ib_spread_batch(st, b->kind_u, tab, map + b->spread_base, 2, (int)ns);
        }));
    if (b->any_flow)
        STEPCHK(timed_b(b, MHD_K_CONTROL, "flow_partial",
                        [&] { return launch_flow_partial_batch(st, b->kind_u, tab, n); }));
    STEPCHK(timed_b(b, MHD_K_CONTROL, "step_end", [&] { return launch_step_end_batch(st, tab, n); }));
    return MHD_OK;
}

// Slot holding the launch tables of the current buffer state (uploaded on first use).
mhd_status current_slot(mhd_batch *b, int *k_out) {
    const std::vector<int> sig = buffer_sig(b);
    for (int k = 0; k < 2; ++k) {
        const BatchSlot &sl = b->slot[k];
        if (sl.valid && sl.version == b->plan_version && sl.sig == sig) {
            *k_out = k;
            return MHD_OK;
        }
    }
    const int k = b->next_slot;
    b->next_slot ^= 1;
    BatchSlot &sl = b->slot[k];
    HIPCHK(hipStreamSynchronize(b->stream));
    if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
    sl.exec = nullptr;
    sl.valid = false;
    std::vector<PipeStep> tab(b->n);
    for (int i = 0; i < b->n; ++i) tab[i] = pipe_step(b->pipes[i]);
    HIPCHK(hipMemcpyAsync(b->tab(k), tab.data(), tab.size() * sizeof(PipeStep), hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipStreamSynchronize(b->stream));
    sl.sig = sig;
    sl.version = b->plan_version;
    sl.valid = true;
    *k_out = k;
    return MHD_OK;
}

mhd_status capture_slot(mhd_batch *b, int k) {
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
    const mhd_status st = issue_step(b, k);
    const hipError_t e = hipStreamEndCapture(b->stream, &graph);
    if (st != MHD_OK) {
        if (e == hipSuccess && graph) (void)hipGraphDestroy(graph);
        return st;
    }
    if (e != hipSuccess) return fail(MHD_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(MHD_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
    b->slot[k].exec = exec;
    return MHD_OK;
}

// Time of `reps` batched sweep rounds over every box (round 0: reads b, writes the scratch copy,
// so the state is unchanged) with the current tiles.
mhd_status time_sweep_round(mhd_batch *b, int reps, hipEvent_t e0, hipEvent_t e1, float *ms) {
    batch_touch(b);
    STEPCHK(build_plan(b));
    int k = 0;
    STEPCHK(current_slot(b, &k));
    auto round = [&]() -> hipError_t {
        for (const auto &g : b->groups) {
            hipError_t e = launch_mag_sweep_batch(b->stream, b->kinds, g.L, b->tab(k), b->map() + g.map_base, 0,
                                                  (int)g.cum.back());
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    HIPCHK(round());  // warm-up
    HIPCHK(hipEventRecord(e0, b->stream));
    for (int r = 0; r < reps; ++r) HIPCHK(round());
    HIPCHK(hipEventRecord(e1, b->stream));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    return MHD_OK;
}

// Autotuner: boxes are grouped by nx (the tile choice depends mostly on the row length); for
// each group in turn every valid tile choice is tried with the other groups fixed, timing the
// whole batched sweep round, and the fastest is kept. Two passes; it starts from the current
// choice, so the result is never slower than that as measured.
mhd_status tune_batch(mhd_batch *b, int reps, hipEvent_t e0, hipEvent_t e1) {
    std::map<int, std::vector<int>> cls;
    for (int i = 0; i < b->n; ++i) cls[b->pipes[i]->g.nx].push_back(i);
    float best = 0.f;
    STEPCHK(time_sweep_round(b, reps, e0, e1, &best));
    for (int pass = 0; pass < 2; ++pass) {
        for (auto &kv : cls) {
            const int nx = kv.first;
            int nz_max = 1;
            for (int i : kv.second) nz_max = std::max(nz_max, b->pipes[i]->g.nz);
            std::vector<SweepLaunch> cand;
            for (int zc : {4, 8, 16}) {
                if (zc > 2 * nz_max && zc != 4) continue;
                if (nx % 128 == 0)
                    for (int ty : {4, 8}) cand.push_back({64, ty, zc, 1});
                for (int tx : {64, 32, 16, 8})
                    if (tx <= std::max(8, nx)) cand.push_back({tx, 4, zc, 0});
            }
            const SweepLaunch keep = b->pipes[kv.second[0]]->sweep;
            SweepLaunch best_L = keep;
            for (const SweepLaunch &L : cand) {
                for (int i : kv.second) b->pipes[i]->sweep = L;
                float ms = 0.f;
                STEPCHK(time_sweep_round(b, reps, e0, e1, &ms));
                if (ms < best) {
                    best = ms;
                    best_L = L;
                }
            }
            for (int i : kv.second) b->pipes[i]->sweep = best_L;
        }
    }
    return MHD_OK;
}

void free_batch(mhd_batch *b) {
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (int k = 0; k < MHD_K_COUNT; ++k)
        for (auto &e : b->ev_pool[k]) {
            (void)hipEventDestroy(e.a);
            (void)hipEventDestroy(e.b);
        }
    for (auto *s : b->pipes) {
        s->owner = nullptr;
        (void)mhd_destroy(s);
    }
    delete b;
}

}  // namespace

extern "C" {

mhd_status mhd_get_tiles(mhd_sim *s, int32_t tiles[4]) {
    g_err.clear();
    if (!s || !tiles) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    tiles[0] = s->sweep.tx;
    tiles[1] = s->sweep.zchunk;
    tiles[2] = s->sweep.pair;
    tiles[3] = s->sweep.ty >= 8 ? 8 : 4;
    return MHD_OK;
}

mhd_status mhd_set_tiles(mhd_sim *s, const int32_t tiles[4]) {
    g_err.clear();
    if (!s || !tiles) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (!valid_tx(tiles[0])) return fail(MHD_ERR_INVALID_ARG, "x tile %d not in {8, 16, 32, 64}", tiles[0]);
    if (tiles[1] < 1) return fail(MHD_ERR_INVALID_ARG, "z chunk must be >= 1");
    if (tiles[2] != 0 && tiles[2] != 1) return fail(MHD_ERR_INVALID_ARG, "paired form flag must be 0 or 1");
    if (tiles[3] != 4 && tiles[3] != 8) return fail(MHD_ERR_INVALID_ARG, "rows of the paired form must be 4 or 8");
    s->sweep.tx = tiles[0];
    s->sweep.zchunk = tiles[1];
    s->sweep.pair = tiles[2];
    s->sweep.ty = tiles[3];
    drop_step_graphs(s);
    if (s->owner) batch_touch(s->owner);
    return MHD_OK;
}

mhd_status mhd_batch_workspace_size(const mhd_pipe_desc *pipes, int32_t n, size_t *bytes) {
    g_err.clear();
    STEPCHK(check_pipes(pipes, n));
    if (!bytes) return fail(MHD_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = make_batch_layout(pipes, n).total;
    return MHD_OK;
}

mhd_status mhd_batch_create(const mhd_pipe_desc *pipes, int32_t n, void *dev_workspace, size_t bytes,
                            void *hip_stream, mhd_batch **out) {
    g_err.clear();
    if (!out) return fail(MHD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    STEPCHK(check_pipes(pipes, n));
    if (!dev_workspace) return fail(MHD_ERR_INVALID_ARG, "device workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % 256) return fail(MHD_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    const BatchLayout L = make_batch_layout(pipes, n);
    if (bytes < L.total) return fail(MHD_ERR_OOM, "workspace has %zu bytes, %zu needed", bytes, L.total);
    mhd_batch *b = new (std::nothrow) mhd_batch();
    if (!b) return fail(MHD_ERR_OOM, "host allocation failed");
    b->n = n;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->ws = static_cast<char *>(dev_workspace);
    b->L = L;
    b->graph = b->stream != nullptr;
    const mhd_grid_desc &g0 = pipes[0].grid;
    b->kinds = pack_kinds(g0.rho_storage, g0.u_storage, g0.b_storage);
    b->kind_u = g0.u_storage;
    b->kind_b = g0.b_storage;
    for (int i = 0; i < n; ++i) {
        mhd_sim *s = nullptr;
        const mhd_status st = mhd_create(&pipes[i].grid, pipes[i].n_markers, b->ws + L.pipe[i], L.pipe_bytes[i],
                                         hip_stream, &s);
        if (st != MHD_OK) {
            const std::string msg = g_err;
            free_batch(b);
            return fail(st, "pipe %d: %s", i, msg.c_str());
        }
        s->owner = b;
        b->pipes.push_back(s);
    }
    *out = b;
    return MHD_OK;
}

mhd_status mhd_batch_pipe(mhd_batch *b, int32_t i, mhd_sim **out) {
    g_err.clear();
    if (!b || !out) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (i < 0 || i >= b->n) return fail(MHD_ERR_INVALID_ARG, "pipe %d outside [0, %d)", i, b->n);
    *out = b->pipes[i];
    return MHD_OK;
}

mhd_status mhd_batch_tune(mhd_batch *b, int32_t reps) {
    g_err.clear();
    if (!b) return fail(MHD_ERR_INVALID_ARG, "batch is NULL");
    if (reps <= 0) reps = 5;
    for (int i = 0; i < b->n; ++i)
        if (!b->pipes[i]->have_params) return fail(MHD_ERR_STATE, "pipe %d has no parameters (mhd_set_params)", i);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    mhd_status st = tune_batch(b, reps, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    batch_touch(b);
    return st;
}

mhd_status mhd_batch_step(mhd_batch *b, int64_t n_steps, int32_t budget_every) {
    g_err.clear();
    if (!b) return fail(MHD_ERR_INVALID_ARG, "batch is NULL");
    if (n_steps < 0) return fail(MHD_ERR_INVALID_ARG, "n_steps < 0");
    if (n_steps == 0) return MHD_OK;
    if (b->plan_version != b->version) STEPCHK(build_plan(b));
    const bool use_graph = b->graph && !b->prof && b->stream != nullptr;
    for (int64_t i = 0; i < n_steps; ++i) {
        int k = 0;
        STEPCHK(current_slot(b, &k));
        if (use_graph) {
            if (!b->slot[k].exec) STEPCHK(capture_slot(b, k));
            HIPCHK(hipGraphLaunch(b->slot[k].exec, b->stream));
        } else {
            STEPCHK(issue_step(b, k));
        }
        for (auto *s : b->pipes) {
            if (s->prm.n_mag & 1) s->cb = 1 - s->cb;
            if (s->split()) s->ch = 1 - s->ch;
            s->cr = 1 - s->cr;
            s->cu = 1 - s->cu;
            s->t_host += 1;
        }
        if (budget_every > 0)
            for (auto *s : b->pipes)
                if (s->t_host % budget_every == 0) STEPCHK(record_budget(s));
    }
    return MHD_OK;
}

mhd_status mhd_batch_set_graph(mhd_batch *b, int32_t enable) {
    g_err.clear();
    if (!b) return fail(MHD_ERR_INVALID_ARG, "batch is NULL");
    if (enable && !b->stream) return fail(MHD_ERR_INVALID_ARG, "graphs need a non-NULL stream");
    b->graph = enable != 0;
    return MHD_OK;
}

mhd_status mhd_batch_set_profiling(mhd_batch *b, int32_t enable) {
    g_err.clear();
    if (!b) return fail(MHD_ERR_INVALID_ARG, "batch is NULL");
    b->prof = enable != 0;
    return MHD_OK;
}

mhd_status mhd_batch_kernel_stats(mhd_batch *b, int32_t kernel, int64_t *launches, double *total_ms) {
    g_err.clear();
    if (!b || !launches || !total_ms) return fail(MHD_ERR_INVALID_ARG, "NULL argument");
    if (kernel < 0 || kernel >= MHD_K_COUNT) return fail(MHD_ERR_INVALID_ARG, "unknown kernel id %d", kernel);
    HIPCHK(hipStreamSynchronize(b->stream));
    double tot = 0.0;
    for (size_t i = 0; i < b->ev_used[kernel]; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, b->ev_pool[kernel][i].a, b->ev_pool[kernel][i].b));
        tot += ms;
    }
    *launches = (int64_t)b->ev_used[kernel];
    *total_ms = tot;
    b->ev_used[kernel] = 0;
    return MHD_OK;
}

mhd_status mhd_batch_destroy(mhd_batch *b) {
    g_err.clear();
    if (!b) return MHD_OK;
    free_batch(b);
    return MHD_OK;
}

}  // extern "C"
