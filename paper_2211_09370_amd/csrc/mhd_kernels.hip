// gfx950 kernels of the single-step simplified lattice Boltzmann step for quasi-static MHD pipe
// flow (arXiv:2211.09370). All arithmetic is float32 except the budget / flow-rate reductions,
// which convert the stored values to float64 and sum them in a fixed order.
//
// Field layout: component-major, x fastest; element (a, x, y, z) at a*N + x + nx*(y + ny*z).
// Storage kinds: float32, or 16-bit offsets (rho - 1 in every kind, u / u_scale, b / b_scale).
//
// Kernels (per fluid step, in order):
//   k_ctrl_begin   body force G(t) of the step (Sec. 4, variable-force form)
//   k_mag_sweep    x n_mag: b*(x) = sum_i g_i^eq(x - e_i), tau_m = 1, c = 6 eta (Sec. 5.7)
//   k_ib_interp    per marker: delta_j = s_j (b_wall - sum_k D_jk phi_k)     (Sec. 5.4 / 5.6)
//   k_ib_spread    per wall-band cell: phi_k += sum_j D_jk delta_j (gather form, no atomics)
//   k_lorentz      F = G x + (curl b) x (B_ext + b), isotropic differences    (Sec. 5.1)
//   k_fluid        single-step rho, rho u with GZS forcing + discrete-effect term (Sec. 3.3, 5.1)
//   k_ib_interp / k_ib_spread on u                                              (Sec. 5.3 / 5.5)
//   k_flow_partial + k_step_end   flow-rate control sum (float64), step counter
//   k_budget_partial + k_budget_final   every K steps: energy budgets of Sec. 4 (float64)
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mhd_internal.h"

namespace mhd {

// -------------------------------------------------------------------------------------------
// Storage traits
// -------------------------------------------------------------------------------------------
template <typename T>
struct St;
// cvt: stored value -> float; from: float times inverse scale -> stored value (float32 storage
// ignores the scale, which is 1 there).
template <>
struct St<float> {
    static __device__ __forceinline__ float ld(const float *p, int64_t i) { return p[i]; }
    static __device__ __forceinline__ void st(float *p, int64_t i, float v) { p[i] = v; }
    static __device__ __forceinline__ float cvt(float v) { return v; }
    static __device__ __forceinline__ float val(float v, float) { return v; }
    static __device__ __forceinline__ float from(float v, float) { return v; }
};
template <>
struct St<__half> {
    static __device__ __forceinline__ float ld(const __half *p, int64_t i) { return __half2float(p[i]); }
    static __device__ __forceinline__ void st(__half *p, int64_t i, float v) { p[i] = __float2half_rn(v); }
    static __device__ __forceinline__ float cvt(__half v) { return __half2float(v); }
    static __device__ __forceinline__ float val(__half v, float scale) { return __half2float(v) * scale; }
    static __device__ __forceinline__ __half from(float v, float inv) { return __float2half_rn(v * inv); }
};
template <>
struct St<__hip_bfloat16> {
    static __device__ __forceinline__ float ld(const __hip_bfloat16 *p, int64_t i) {
        return __bfloat162float(p[i]);
    }
    static __device__ __forceinline__ void st(__hip_bfloat16 *p, int64_t i, float v) {
        p[i] = __float2bfloat16(v);
    }
    static __device__ __forceinline__ float cvt(__hip_bfloat16 v) { return __bfloat162float(v); }
    static __device__ __forceinline__ float val(__hip_bfloat16 v, float scale) { return __bfloat162float(v) * scale; }
    static __device__ __forceinline__ __hip_bfloat16 from(float v, float inv) { return __float2bfloat16(v * inv); }
};

// Element at a 32-bit byte offset from a wave-uniform base: lets the compiler use the
// scalar-base + 32-bit vector-offset addressing form instead of 64-bit address arithmetic.
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, unsigned byte_off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_off(T *base, unsigned byte_off, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off) = v;
}

__device__ __forceinline__ int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// D3Q19 neighbour offsets without the rest direction: 6 faces (w = 1/18), 12 edges (w = 1/36).
__constant__ int c_dir[18][3] = {{1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                                 {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1},
                                 {1, 0, -1}, {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
#define W0 (1.0f / 3.0f)
#define WF (1.0f / 18.0f)
#define WE (1.0f / 36.0f)

// -------------------------------------------------------------------------------------------
// Control kernels
// -------------------------------------------------------------------------------------------
__device__ __forceinline__ void ctrl_begin_body(DevCtrl *ctrl, const StepConst &c) {
    double G;
    if (c.flow_control)
        G = ctrl->G;
    else if (c.period > 0.0)
        G = c.G0 + c.G1 * cos(2.0 * 3.14159265358979323846 * (double)ctrl->t / c.period);
    else
        G = c.G0;
    ctrl->G_step = G;
}
__global__ void k_ctrl_begin(DevCtrl *ctrl, StepConst c) {
    if (threadIdx.x == 0) ctrl_begin_body(ctrl, c);
}
// one workgroup per box
__global__ void k_ctrl_begin_batch(const PipeStep *tab) {
    if (threadIdx.x == 0) ctrl_begin_body(tab[blockIdx.x].ctrl, tab[blockIdx.x].c);
}

// Fixed-order sum of the flow partials (one block per box), integral control law, step counter.
template <bool BATCH>
__global__ void __launch_bounds__(kRedThreads) k_step_end(DevCtrl *ctrl, const double *part, StepConst c,
                                                          double inv_count, const PipeStep *tab) {
    if constexpr (BATCH) {
        const PipeStep &q = tab[blockIdx.x];
        ctrl = q.ctrl;
        part = q.flow_part;
        c = q.c;
        inv_count = q.inv_count;
    }
    __shared__ double sh[kRedThreads];
    double s = 0.0;
    if (c.flow_control)
        for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (c.flow_control) {
            double ub = sh[0] * inv_count;
            ctrl->G = ctrl->G + c.k_c * (8.0 * c.nu / (c.radius * c.radius)) * (c.u_target - ub);
        } else {
            ctrl->G = ctrl->G_step;
        }
        ctrl->t += 1;
    }
}

__global__ void k_reset_records(DevCtrl *ctrl) {
    if (threadIdx.x == 0) {
        ctrl->n_records = 0;
        ctrl->overflow = 0;
    }
}

// -------------------------------------------------------------------------------------------
// Magnetic sweep (Sec. 5.7): tau_m = 1, particle speed c = 6 eta, so c_i / c_s^2 = e_i / (2 eta).
//
//   b*_a(x) = sum_i w_i [ b_a(x - e_i) + kappa sum_c e_ic Lam_ac(x - e_i) ],
//   Lam_ac = u_c B_a - u_a B_c,  B = B_ext + b,  kappa = 1 / (2 eta).
//
// Written per plane: a workgroup owns a TX x TY column of cells and marches along z over a
// chunk of planes. Each new plane (with a one-cell x/y halo) is staged in LDS as
// (b_x, b_y, b_z, kappa Lam_xy, kappa Lam_xz, kappa Lam_yz); every thread forms from its 3x3
// in-plane neighbourhood the plane's contributions to the outputs at z-1, z and z+1
// (A, B, C below) and keeps the running sums in registers, so each field value is read from
// memory once per plane and every neighbour access is an LDS read.
//
// With D_c[f](x) = sum_i w_i e_ic f(x - e_i) and the in-plane sums
//   P0 = c/3 + (faces)/18 + (corners)/36,  P1 = c/18 + (faces)/36,
//   Q0x = (xm - xp)/18 + (mm + mp - pm - pp)/36,  Q1x = (xm - xp)/36   (Q*y likewise in y),
// one has avg[f](z) = P0(z) + P1(z-1) + P1(z+1), D_x[f](z) = Q0x(z) + Q1x(z-1) + Q1x(z+1),
// D_y likewise and D_z[f](z) = P1(z-1) - P1(z+1); then
//   b*_x = avg b_x + D_y Lxy + D_z Lxz,  b*_y = avg b_y - D_x Lxy + D_z Lyz,
//   b*_z = avg b_z - D_x Lxz - D_y Lyz.
// -------------------------------------------------------------------------------------------
template <int TX, int TY, typename TU, typename TB, bool BATCH>
__global__ void __launch_bounds__(TX *TY) k_mag_sweep(SweepArgs a, const PipeStep *tab, const BlockMap *map,
                                                      int parity, int nbatch) {
    constexpr int NT = TX * TY, HX = TX + 2, HY = TY + 2, HN = HX * HY;
    constexpr int NSLOT = (HN + NT - 1) / NT;
    // two LDS planes: the next plane is staged while the current one is reduced
    __shared__ float s_pl[2][6][HN];

    // XCD-aware order: the hardware hands consecutive workgroups to the 8 XCDs in turn; give
    // each XCD a contiguous run of tiles so neighbouring tiles share halo rows in one L2.
    const int per = gridDim.x >> 3;
    int lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if constexpr (BATCH) {
        if (lb >= nbatch) return;
        const BlockMap m = map[lb];
        a = tab[m.pipe].sw[parity];
        lb = m.local;
    } else {
        if (lb >= a.nblocks) return;
    }
    const int tix = lb % a.tiles_x;
    const int rest = lb / a.tiles_x;
    const int tiy = rest % a.tiles_y;
    const int tiz = rest / a.tiles_y;
    const int x0 = tix * TX, y0 = tiy * TY;
    const int z0 = tiz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned N = (unsigned)nx * ny * nz;  // 3 N < 2^31: 32-bit offsets from uniform bases
    const unsigned plane = (unsigned)nx * ny;

    const TU *u0 = (const TU *)a.u, *u1 = u0 + N, *u2 = u0 + 2 * (size_t)N;
    const TB *b0 = (const TB *)a.b, *b1 = b0 + N, *b2 = b0 + 2 * (size_t)N;
    TB *o0 = (TB *)a.bo, *o1 = o0 + N, *o2 = o0 + 2 * (size_t)N;

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool own = gx < nx && gy < ny;

    // halo slots handled by this thread: fixed (x, y) for the whole march
    unsigned sxy[NSLOT];
    float sbe[NSLOT][3];
    bool sval[NSLOT];
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
        const int i = tid + s * NT;
        sval[s] = i < HN;
        const int hx = i % HX, hy = i / HX;
        const int hxg = wrapi(x0 - 1 + hx, nx), hyg = wrapi(y0 - 1 + hy, ny);
        sxy[s] = (unsigned)(hxg + nx * hyg);
        sbe[s][0] = sval[s] ? a.bext[hxg] : 0.f;
        sbe[s][1] = sval[s] ? a.bext[nx + hxg] : 0.f;
        sbe[s][2] = sval[s] ? a.bext[2 * nx + hxg] : 0.f;
    }

    // raw stored values of the next plane: converted only when they are written to LDS, so the
    // loads stay in flight while the current plane is reduced
    TU ru[NSLOT][3];
    TB rb[NSLOT][3];
    auto load_plane = [&](int p) {
        const unsigned off = (unsigned)wrapi(p, nz) * plane;
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            if (sval[s]) {
                const unsigned ku = (off + sxy[s]) * (unsigned)sizeof(TU);
                const unsigned kb = (off + sxy[s]) * (unsigned)sizeof(TB);
                ru[s][0] = ld_off(u0, ku);
                ru[s][1] = ld_off(u1, ku);
                ru[s][2] = ld_off(u2, ku);
                rb[s][0] = ld_off(b0, kb);
                rb[s][1] = ld_off(b1, kb);
                rb[s][2] = ld_off(b2, kb);
            }
        }
    };

    const int c0 = (ly + 1) * HX + (lx + 1);
    const float kap = a.kappa;
    constexpr float W6 = 1.0f / 6.0f;  // WF + 4 WE: weight of a neighbouring plane as a whole
    // running sums of the plane contributions (difference form), and the column's own values
    float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
    float ap0 = 0.f, ap1 = 0.f, ap2 = 0.f;
    float cm0 = 0.f, cm1 = 0.f, cm2 = 0.f;  // b at (x, y, z-1)
    float cc0 = 0.f, cc1 = 0.f, cc2 = 0.f;  // b at (x, y, z)

    // stage the raw values in the registers into LDS buffer S as (b, kappa Lam)
    auto stage = [&](auto buf) {
        constexpr int S = decltype(buf)::value;
#pragma unroll
        for (int s = 0; s < NSLOT; ++s) {
            if (sval[s]) {
                const int i = tid + s * NT;
                const float bx = St<TB>::val(rb[s][0], a.b_scale);
                const float by = St<TB>::val(rb[s][1], a.b_scale);
                const float bz = St<TB>::val(rb[s][2], a.b_scale);
                const float Bx = bx + sbe[s][0];
                const float By = by + sbe[s][1];
                const float Bz = bz + sbe[s][2];
                const float ux = St<TU>::val(ru[s][0], a.u_scale);
                const float uy = St<TU>::val(ru[s][1], a.u_scale);
                const float uz = St<TU>::val(ru[s][2], a.u_scale);
                s_pl[S][0][i] = bx;
                s_pl[S][1][i] = by;
                s_pl[S][2][i] = bz;
                s_pl[S][3][i] = kap * (uy * Bx - ux * By);
                s_pl[S][4][i] = kap * (uz * Bx - ux * Bz);
                s_pl[S][5][i] = kap * (uz * By - uy * Bz);
            }
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;

    // plane r = p - (z0 - 1) is reduced from LDS buffer r % 2; while it is, the next plane is
    // staged into the other buffer and the one after that is requested into the registers
    load_plane(z0 - 1);
    stage(I0{});
    load_plane(z0);
    __syncthreads();
    auto body = [&](auto par, int p) {
        constexpr int P = decltype(par)::value;  // parity of plane p
        using Q = std::integral_constant<int, 1 - P>;
        // plane p+1 goes from the registers to the other LDS buffer (its last readers passed
        // the previous barrier); the registers then request plane p+2
        if (p < z1) {
            stage(Q{});
            if (p + 2 <= z1) load_plane(p + 2);
        }
        const int cur = P;
        const float *s_bx = s_pl[cur][0], *s_by = s_pl[cur][1], *s_bz = s_pl[cur][2];
        const float *s_lxy = s_pl[cur][3], *s_lxz = s_pl[cur][4], *s_lyz = s_pl[cur][5];
        if (own) {
            // b components: centre value and in-plane sums of differences to it
            //   dP0 = sum_faces WF (f - c) + sum_corners WE (f - c),  dP1 = sum_faces WE (f - c)
            float c_x, c_y, c_z, dP0x, dP1x, dP0y, dP1y, dP0z, dP1z;
#define MHD_PLANE_DIFFS(F, C, DP0, DP1)                                                              \
    {                                                                                                \
        const float *f = F;                                                                          \
        C = f[c0];                                                                                   \
        const float fs = ((f[c0 - 1] - C) + (f[c0 + 1] - C)) + ((f[c0 - HX] - C) + (f[c0 + HX] - C)); \
        const float cs = ((f[c0 - HX - 1] - C) + (f[c0 - HX + 1] - C)) +                              \
                         ((f[c0 + HX - 1] - C) + (f[c0 + HX + 1] - C));                               \
        DP0 = WF * fs + WE * cs;                                                                     \
        DP1 = WE * fs;                                                                               \
    }
            MHD_PLANE_DIFFS(s_bx, c_x, dP0x, dP1x)
            MHD_PLANE_DIFFS(s_by, c_y, dP0y, dP1y)
            MHD_PLANE_DIFFS(s_bz, c_z, dP0z, dP1z)
            // kappa Lam_xy: Q0x, Q1x, Q0y, Q1y (differences across the cell)
            float Q0xA, Q1xA, Q0yA, Q1yA;
            {
                const float *f = s_lxy;
                const float dx = f[c0 - 1] - f[c0 + 1], dy = f[c0 - HX] - f[c0 + HX];
                const float mm = f[c0 - HX - 1], pm = f[c0 - HX + 1], mp = f[c0 + HX - 1], pp = f[c0 + HX + 1];
                Q0xA = WF * dx + WE * ((mm - pm) + (mp - pp));
                Q1xA = WE * dx;
                Q0yA = WF * dy + WE * ((mm - mp) + (pm - pp));
                Q1yA = WE * dy;
            }
            // kappa Lam_xz: P1, Q0x, Q1x and kappa Lam_yz: P1, Q0y, Q1y. These flux terms are
            // of order b / R, so plain weighted sums keep their rounding below that of b.
            float P1B, Q0xB, Q1xB;
            {
                const float *f = s_lxz;
                const float xm = f[c0 - 1], xp = f[c0 + 1];
                const float mm = f[c0 - HX - 1], pm = f[c0 - HX + 1], mp = f[c0 + HX - 1], pp = f[c0 + HX + 1];
                P1B = WF * f[c0] + WE * ((xm + xp) + (f[c0 - HX] + f[c0 + HX]));
                Q0xB = WF * (xm - xp) + WE * ((mm - pm) + (mp - pp));
                Q1xB = WE * (xm - xp);
            }
            float P1C, Q0yC, Q1yC;
            {
                const float *f = s_lyz;
                const float ym = f[c0 - HX], yp = f[c0 + HX];
                const float mm = f[c0 - HX - 1], pm = f[c0 - HX + 1], mp = f[c0 + HX - 1], pp = f[c0 + HX + 1];
                P1C = WF * f[c0] + WE * ((f[c0 - 1] + f[c0 + 1]) + (ym + yp));
                Q0yC = WF * (ym - yp) + WE * ((mm - mp) + (pm - pp));
                Q1yC = WE * (ym - yp);
            }
            // contributions of this plane to the outputs at z+1 (A), z (B), z-1 (C)
            const float A0 = dP1x + Q1yA + P1B, B0 = dP0x + Q0yA, C0 = dP1x + Q1yA - P1B;
            const float A1 = dP1y - Q1xA + P1C, B1 = dP0y - Q0xA, C1 = dP1y - Q1xA - P1C;
            const float A2 = dP1z - Q1xB - Q1yC, B2 = dP0z - Q0xB - Q0yC;
            if (p >= z0 + 1) {
                // output plane p-1: b* = b_c + increment, the increment built from differences
                const float d0 = (acc0 + C0) + W6 * ((cm0 - cc0) + (c_x - cc0));
                const float d1 = (acc1 + C1) + W6 * ((cm1 - cc1) + (c_y - cc1));
                const float d2 = (acc2 + A2) + W6 * ((cm2 - cc2) + (c_z - cc2));
                const unsigned k = ((unsigned)(p - 1) * plane + (unsigned)(gx + nx * gy)) * (unsigned)sizeof(TB);
                st_off(o0, k, St<TB>::from(cc0 + d0, a.inv_b_scale));
                st_off(o1, k, St<TB>::from(cc1 + d1, a.inv_b_scale));
                st_off(o2, k, St<TB>::from(cc2 + d2, a.inv_b_scale));
            }
            acc0 = ap0 + B0;
            acc1 = ap1 + B1;
            acc2 = ap2 + B2;
            ap0 = A0;
            ap1 = A1;
            ap2 = A2;
            cm0 = cc0;
            cm1 = cc1;
            cm2 = cc2;
            cc0 = c_x;
            cc1 = c_y;
            cc2 = c_z;
        }
        __syncthreads();  // plane p+1 is staged; buffer `cur` may be overwritten next
    };
    for (int p = z0 - 1; p <= z1; p += 2) {
        body(I0{}, p);
        if (p + 1 <= z1) body(I1{}, p + 1);
    }
#undef MHD_PLANE_DIFFS
}

// -------------------------------------------------------------------------------------------
// Paired magnetic sweep for boxes with n_x a multiple of 128: the same plane march and the same
// per-cell arithmetic as k_mag_sweep, but every lane owns two neighbouring x cells, so a wave
// covers a 128-cell row. Rows are loaded and stored as 8-byte (float32) or 4-byte (16-bit)
// pairs — half the memory instructions per cell — and a lane reads the four values x-1 .. x+2
// of a row from LDS with one 8-byte and two 4-byte reads serving both of its cells.
// -------------------------------------------------------------------------------------------
template <typename T>
struct Pair;
template <>
struct Pair<float> {
    using raw = float2;
    static __device__ __forceinline__ float lo(raw v, float) { return v.x; }
    static __device__ __forceinline__ float hi(raw v, float) { return v.y; }
    static __device__ __forceinline__ raw make(float a, float b, float) { return make_float2(a, b); }
};
template <>
struct Pair<__half> {
    using raw = __half2;
    static __device__ __forceinline__ float lo(raw v, float s) { return __low2float(v) * s; }
    static __device__ __forceinline__ float hi(raw v, float s) { return __high2float(v) * s; }
    static __device__ __forceinline__ raw make(float a, float b, float inv) {
        return __halves2half2(__float2half_rn(a * inv), __float2half_rn(b * inv));
    }
};
template <>
struct Pair<__hip_bfloat16> {
    using raw = unsigned;  // low half = element x, high half = element x + 1
    static __device__ __forceinline__ float lo(raw v, float s) { return __uint_as_float(v << 16) * s; }
    static __device__ __forceinline__ float hi(raw v, float s) { return __uint_as_float(v & 0xffff0000u) * s; }
    static __device__ __forceinline__ raw make(float a, float b, float inv) {
        const __hip_bfloat16 x = __float2bfloat16(a * inv), y = __float2bfloat16(b * inv);
        return (unsigned)__bfloat16_as_ushort(x) | ((unsigned)__bfloat16_as_ushort(y) << 16);
    }
};

template <int TY, typename TU, typename TB, bool BATCH>
__global__ void __launch_bounds__(64 * TY) k_mag_sweep_pair(SweepArgs a, const PipeStep *tab, const BlockMap *map,
                                                            int parity, int nbatch) {
    constexpr int HY = TY + 2;        // staged rows
    constexpr int RS = 132;           // LDS row stride: x0-1 at 0, x0 .. x0+127 at 1 .. 128, x0+128 at 129
    constexpr int NR = (HY + TY - 1) / TY;  // row-load rounds per wave
    __shared__ __align__(16) float s_pl[2][6][HY * RS];

    const int per = gridDim.x >> 3;
    int lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if constexpr (BATCH) {
        if (lb >= nbatch) return;
        const BlockMap m = map[lb];
        a = tab[m.pipe].sw[parity];
        lb = m.local;
    } else {
        if (lb >= a.nblocks) return;
    }
    const int tix = lb % a.tiles_x;
    const int rest = lb / a.tiles_x;
    const int tiy = rest % a.tiles_y;
    const int tiz = rest / a.tiles_y;
    const int x0 = tix * 128, y0 = tiy * TY;
    const int z0 = tiz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, a.nz);
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const unsigned N = (unsigned)nx * ny * nz;
    const unsigned plane = (unsigned)nx * ny;
    const TU *u0 = (const TU *)a.u, *u1 = u0 + N, *u2 = u0 + 2 * (size_t)N;
    const TB *b0 = (const TB *)a.b, *b1 = b0 + N, *b2 = b0 + 2 * (size_t)N;
    TB *o0 = (TB *)a.bo, *o1 = o0 + N, *o2 = o0 + 2 * (size_t)N;
    using PU = Pair<TU>;
    using PB = Pair<TB>;
    using RU = typename PU::raw;
    using RB = typename PB::raw;

    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63;
    const int xa = x0 + 2 * l;            // this lane's cells: xa, xa + 1 (always inside: nx % 128 == 0)
    const int gy = y0 + w;
    const bool own = gy < ny;
    const float kap = a.kappa;
    // B_ext of this lane's pair of columns and of the two halo columns
    const float bea[3] = {a.bext[xa], a.bext[nx + xa], a.bext[2 * nx + xa]};
    const float beb[3] = {a.bext[xa + 1], a.bext[nx + xa + 1], a.bext[2 * nx + xa + 1]};

    // row loads: round r stages row hy = w + r * TY (if < HY) at columns xa, xa + 1
    unsigned rowoff[NR];
    bool rowval[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int hy = w + r * TY;
        rowval[r] = hy < HY;
        rowoff[r] = (unsigned)(xa + nx * wrapi(y0 - 1 + hy, ny));
    }
    // halo columns: lanes 0 .. 2*HY-1 of the last wave, lane -> (row hy = lane / 2, side)
    const bool hval = (w == TY - 1) && (l < 2 * HY);
    const int hhy = l >> 1, hside = l & 1;
    const int hx = hside ? wrapi(x0 + 128, nx) : wrapi(x0 - 1, nx);
    const unsigned hoff = (unsigned)(hx + nx * wrapi(y0 - 1 + min(hhy, HY - 1), ny));
    const int hidx = min(hhy, HY - 1) * RS + (hside ? 129 : 0);
    const float hbe[3] = {a.bext[hx], a.bext[nx + hx], a.bext[2 * nx + hx]};

    RU ru[NR][3];
    RB rb[NR][3];
    TU hu[3];
    TB hb[3];
    auto load_plane = [&](int p) {
        const unsigned off = (unsigned)wrapi(p, nz) * plane;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (rowval[r]) {
                const unsigned ku = (off + rowoff[r]) * (unsigned)sizeof(TU);
                const unsigned kb = (off + rowoff[r]) * (unsigned)sizeof(TB);
                ru[r][0] = ld_off(reinterpret_cast<const RU *>(u0), ku);
                ru[r][1] = ld_off(reinterpret_cast<const RU *>(u1), ku);
                ru[r][2] = ld_off(reinterpret_cast<const RU *>(u2), ku);
                rb[r][0] = ld_off(reinterpret_cast<const RB *>(b0), kb);
                rb[r][1] = ld_off(reinterpret_cast<const RB *>(b1), kb);
                rb[r][2] = ld_off(reinterpret_cast<const RB *>(b2), kb);
            }
        }
        if (hval) {
            const unsigned ku = (off + hoff) * (unsigned)sizeof(TU), kb = (off + hoff) * (unsigned)sizeof(TB);
            hu[0] = ld_off(u0, ku);
            hu[1] = ld_off(u1, ku);
            hu[2] = ld_off(u2, ku);
            hb[0] = ld_off(b0, kb);
            hb[1] = ld_off(b1, kb);
            hb[2] = ld_off(b2, kb);
        }
    };
    auto put = [&](int buf, int idx, float bx, float by, float bz, float ux, float uy, float uz, const float *be) {
        const float Bx = bx + be[0], By = by + be[1], Bz = bz + be[2];
        s_pl[buf][0][idx] = bx;
        s_pl[buf][1][idx] = by;
        s_pl[buf][2][idx] = bz;
        s_pl[buf][3][idx] = kap * (uy * Bx - ux * By);
        s_pl[buf][4][idx] = kap * (uz * Bx - ux * Bz);
        s_pl[buf][5][idx] = kap * (uz * By - uy * Bz);
    };
    auto stage = [&](auto bufc) {
        constexpr int S = decltype(bufc)::value;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (rowval[r]) {
                const int idx = (w + r * TY) * RS + 1 + 2 * l;
                const float us = a.u_scale, bs = a.b_scale;
                put(S, idx, PB::lo(rb[r][0], bs), PB::lo(rb[r][1], bs), PB::lo(rb[r][2], bs), PU::lo(ru[r][0], us),
                    PU::lo(ru[r][1], us), PU::lo(ru[r][2], us), bea);
                put(S, idx + 1, PB::hi(rb[r][0], bs), PB::hi(rb[r][1], bs), PB::hi(rb[r][2], bs), PU::hi(ru[r][0], us),
                    PU::hi(ru[r][1], us), PU::hi(ru[r][2], us), beb);
            }
        }
        if (hval)
            put(S, hidx, St<TB>::val(hb[0], a.b_scale), St<TB>::val(hb[1], a.b_scale), St<TB>::val(hb[2], a.b_scale),
                St<TU>::val(hu[0], a.u_scale), St<TU>::val(hu[1], a.u_scale), St<TU>::val(hu[2], a.u_scale), hbe);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;

    constexpr float W6 = 1.0f / 6.0f;
    float acc[2][3] = {}, ap[2][3] = {}, cm[2][3] = {}, cc[2][3] = {};

    load_plane(z0 - 1);
    stage(I0{});
    load_plane(z0);
    __syncthreads();
    auto body = [&](auto par, int p) {
        constexpr int P = decltype(par)::value;
        using Q = std::integral_constant<int, 1 - P>;
        if (p < z1) {
            stage(Q{});
            if (p + 2 <= z1) load_plane(p + 2);
        }
        if (own) {
            // per field: rows y-1, y, y+1 at columns xa-1 .. xa+2 (two aligned 8-byte reads per
            // row), reduced at once into the plane terms of both cells
            float A[2][3], B[2][3], C[2][2], cen[2][3];
            auto rows = [&](int k, float (&v)[3][4]) {
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const float *row = &s_pl[P][k][(w + r) * RS + 2 * l];
                    const float2 lo = *reinterpret_cast<const float2 *>(row);
                    const float2 hi = *reinterpret_cast<const float2 *>(row + 2);
                    v[r][0] = lo.x;
                    v[r][1] = lo.y;
                    v[r][2] = hi.x;
                    v[r][3] = hi.y;
                }
            };
            {  // b components
                float v[3][4];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    rows(k, v);
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const float c = v[1][1 + e];
                        const float fs = ((v[1][e] - c) + (v[1][e + 2] - c)) + ((v[0][1 + e] - c) + (v[2][1 + e] - c));
                        const float cs = ((v[0][e] - c) + (v[0][e + 2] - c)) + ((v[2][e] - c) + (v[2][e + 2] - c));
                        const float dP0 = WF * fs + WE * cs, dP1 = WE * fs;
                        cen[e][k] = c;
                        A[e][k] = dP1;
                        B[e][k] = dP0;
                        if (k < 2) C[e][k] = dP1;
                    }
                }
            }
            {  // kappa Lam_xy: Q0x, Q1x, Q0y, Q1y
                float v[3][4];
                rows(3, v);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float dx = v[1][e] - v[1][e + 2], dy = v[0][1 + e] - v[2][1 + e];
                    const float Q0x = WF * dx + WE * ((v[0][e] - v[0][e + 2]) + (v[2][e] - v[2][e + 2]));
                    const float Q1x = WE * dx;
                    const float Q0y = WF * dy + WE * ((v[0][e] - v[2][e]) + (v[0][e + 2] - v[2][e + 2]));
                    const float Q1y = WE * dy;
                    A[e][0] += Q1y;
                    B[e][0] += Q0y;
                    C[e][0] += Q1y;
                    A[e][1] -= Q1x;
                    B[e][1] -= Q0x;
                    C[e][1] -= Q1x;
                }
            }
            {  // kappa Lam_xz: P1, Q0x, Q1x
                float v[3][4];
                rows(4, v);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float dx = v[1][e] - v[1][e + 2];
                    const float P1 = WF * v[1][1 + e] + WE * ((v[1][e] + v[1][e + 2]) + (v[0][1 + e] + v[2][1 + e]));
                    const float Q0x = WF * dx + WE * ((v[0][e] - v[0][e + 2]) + (v[2][e] - v[2][e + 2]));
                    const float Q1x = WE * dx;
                    A[e][0] += P1;
                    C[e][0] -= P1;
                    A[e][2] -= Q1x;
                    B[e][2] -= Q0x;
                }
            }
            {  // kappa Lam_yz: P1, Q0y, Q1y
                float v[3][4];
                rows(5, v);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float dy = v[0][1 + e] - v[2][1 + e];
                    const float P1 = WF * v[1][1 + e] + WE * ((v[1][e] + v[1][e + 2]) + (v[0][1 + e] + v[2][1 + e]));
                    const float Q0y = WF * dy + WE * ((v[0][e] - v[2][e]) + (v[0][e + 2] - v[2][e + 2]));
                    const float Q1y = WE * dy;
                    A[e][1] += P1;
                    C[e][1] -= P1;
                    A[e][2] -= Q1y;
                    B[e][2] -= Q0y;
                }
            }
            float out[2][3];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                // output plane p-1: b* = b_c + increment (differences only); C2 = A2
                out[e][0] = cc[e][0] + ((acc[e][0] + C[e][0]) + W6 * ((cm[e][0] - cc[e][0]) + (cen[e][0] - cc[e][0])));
                out[e][1] = cc[e][1] + ((acc[e][1] + C[e][1]) + W6 * ((cm[e][1] - cc[e][1]) + (cen[e][1] - cc[e][1])));
                out[e][2] = cc[e][2] + ((acc[e][2] + A[e][2]) + W6 * ((cm[e][2] - cc[e][2]) + (cen[e][2] - cc[e][2])));
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    acc[e][q] = ap[e][q] + B[e][q];
                    ap[e][q] = A[e][q];
                    cm[e][q] = cc[e][q];
                    cc[e][q] = cen[e][q];
                }
            }
            if (p >= z0 + 1) {
                const unsigned k = ((unsigned)(p - 1) * plane + (unsigned)(xa + nx * gy)) * (unsigned)sizeof(TB);
                st_off(reinterpret_cast<RB *>(o0), k, PB::make(out[0][0], out[1][0], a.inv_b_scale));
                st_off(reinterpret_cast<RB *>(o1), k, PB::make(out[0][1], out[1][1], a.inv_b_scale));
                st_off(reinterpret_cast<RB *>(o2), k, PB::make(out[0][2], out[1][2], a.inv_b_scale));
            }
        }
        __syncthreads();
    };
    for (int p = z0 - 1; p <= z1; p += 2) {
        body(I0{}, p);
        if (p + 1 <= z1) body(I1{}, p + 1);
    }
}

// -------------------------------------------------------------------------------------------
// Immersed boundary (Sec. 5.2 - 5.6), explicit diagonal form:
//   delta_j = s_j (phi_wall_j - sum_k D_jk phi*_k),  phi_k = phi*_k + sum_j D_jk delta_j,
// s_j = lambda / (d_j (1 + d_j (lambda - 1))).
// Two launches: every interpolation (per marker, to delta in memory) is taken before any cell
// changes (per wall-band cell gather, no atomics, entries in marker order). Taps of a marker
// and entries of a cell are padded to fixed counts (weight 0) and stored structure-of-arrays,
// so all loads of a thread are independent. Markers are ordered by the (y, z) of their stencil
// and then by x, band cells by cell index: neighbouring lanes of a wave then address
// neighbouring x, i.e. consecutive words of the x-fastest fields.
// -------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void ib_marker(const T *phi, float scale, const IbArgs &a, int j, float &d0, float &d1,
                                          float &d2) {
    float I0 = 0.f, I1 = 0.f, I2 = 0.f;
#pragma unroll 9
    for (int t = 0; t < a.tm; ++t) {
        const int64_t k = a.tap_cell[(int64_t)t * a.M + j];
        const float w = a.tap_w[(int64_t)t * a.M + j];
        I0 += w * (St<T>::ld(phi, k) * scale);
        I1 += w * (St<T>::ld(phi, a.N + k) * scale);
        I2 += w * (St<T>::ld(phi, 2 * a.N + k) * scale);
    }
    const float s = a.sj[j];
    d0 = s * (a.wall[j] - I0);
    d1 = s * (a.wall[a.M + j] - I1);
    d2 = s * (a.wall[2 * a.M + j] - I2);
}

template <typename T>
__device__ __forceinline__ void ib_cell(T *phi, float scale, float inv_scale, const IbArgs &a, int e,
                                        const float *d0, const float *d1, const float *d2, int base) {
    const int64_t k = a.band_cell[e];
    const float v0 = St<T>::ld(phi, k) * scale, v1 = St<T>::ld(phi, a.N + k) * scale,
                v2 = St<T>::ld(phi, 2 * a.N + k) * scale;
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
#pragma unroll 4
    for (int q = 0; q < a.km; ++q) {
        const int j = a.band_mk[(int64_t)q * a.nband + e] - base;
        const float w = a.band_w[(int64_t)q * a.nband + e];
        c0 += w * d0[j];
        c1 += w * d1[j];
        c2 += w * d2[j];
    }
    St<T>::st(phi, k, (v0 + c0) * inv_scale);
    St<T>::st(phi, a.N + k, (v1 + c1) * inv_scale);
    St<T>::st(phi, 2 * a.N + k, (v2 + c2) * inv_scale);
}

template <typename T, bool BATCH>
__global__ void __launch_bounds__(kIbThreads) k_ib_interp(const T *phi, float scale, IbArgs a, const PipeStep *tab,
                                                          const BlockMap *map, int which) {
    int blk = blockIdx.x;
    if constexpr (BATCH) {
        const BlockMap m = map[blk];
        const PipeStep &q = tab[m.pipe];
        a = q.ib[which];
        phi = (const T *)q.phi[which];
        scale = q.scale[which];
        blk = m.local;
    }
    const int j = blk * kIbThreads + threadIdx.x;
    if (j >= a.M) return;
    float d0, d1, d2;
    ib_marker(phi, scale, a, j, d0, d1, d2);
    a.delta[j] = d0;
    a.delta[a.M + j] = d1;
    a.delta[2 * a.M + j] = d2;
}

template <typename T, bool BATCH>
__global__ void __launch_bounds__(kIbThreads) k_ib_spread(T *phi, float scale, float inv_scale, IbArgs a,
                                                          const PipeStep *tab, const BlockMap *map, int which) {
    int blk = blockIdx.x;
    if constexpr (BATCH) {
        const BlockMap m = map[blk];
        const PipeStep &q = tab[m.pipe];
        a = q.ib[which];
        phi = (T *)q.phi[which];
        scale = q.scale[which];
        inv_scale = q.inv_scale[which];
        blk = m.local;
    }
    const int e = blk * kIbThreads + threadIdx.x;
    if (e >= a.nband) return;
    ib_cell(phi, scale, inv_scale, a, e, a.delta, a.delta + a.M, a.delta + 2 * a.M, 0);
}

// -------------------------------------------------------------------------------------------
// Lorentz + body force (Sec. 5.1): J = curl_h b with d_a f = 3 sum_i w_i e_ia f(x + e_i),
// F = G x + J x (B_ext + b).
// -------------------------------------------------------------------------------------------
template <typename TB, bool BATCH>
__global__ void __launch_bounds__(kCellThreads) k_lorentz(const TB *b, float bs, const float *bext,
                                                          const DevCtrl *ctrl, float *F, StepConst c,
                                                          const PipeStep *tab, const BlockMap *map) {
    int64_t blk = blockIdx.x;
    if constexpr (BATCH) {
        const BlockMap m = map[blk];
        const PipeStep &q = tab[m.pipe];
        b = (const TB *)q.b_last;
        bs = q.c.b_scale;
        bext = q.bext;
        ctrl = q.ctrl;
        F = q.F;
        c = q.c;
        blk = m.local;
    }
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    const int64_t k = blk * kCellThreads + threadIdx.x;
    if (k >= N) return;
    const int x = (int)(k % c.nx);
    const int y = (int)((k / c.nx) % c.ny);
    const int z = (int)(k / ((int64_t)c.nx * c.ny));
    float g[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};  // g[a][c] = d_c b_a
#pragma unroll
    for (int i = 0; i < 18; ++i) {
        const int ex = c_dir[i][0], ey = c_dir[i][1], ez = c_dir[i][2];
        const float w = 3.0f * (i < 6 ? WF : WE);
        const int64_t kn = wrapi(x + ex, c.nx) + (int64_t)c.nx * (wrapi(y + ey, c.ny) + (int64_t)c.ny * wrapi(z + ez, c.nz));
        const float v0 = St<TB>::ld(b, kn) * bs, v1 = St<TB>::ld(b, N + kn) * bs, v2 = St<TB>::ld(b, 2 * N + kn) * bs;
        const float e3[3] = {(float)ex, (float)ey, (float)ez};
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            const float we = w * e3[cc];
            g[0][cc] += we * v0;
            g[1][cc] += we * v1;
            g[2][cc] += we * v2;
        }
    }
    const float Jx = g[2][1] - g[1][2], Jy = g[0][2] - g[2][0], Jz = g[1][0] - g[0][1];
    const float Bx = St<TB>::ld(b, k) * bs + bext[x];
    const float By = St<TB>::ld(b, N + k) * bs + bext[c.nx + x];
    const float Bz = St<TB>::ld(b, 2 * N + k) * bs + bext[2 * c.nx + x];
    const float G = (float)ctrl->G_step;
    F[k] = G + (Jy * Bz - Jz * By);
    F[N + k] = Jz * Bx - Jx * Bz;
    F[2 * N + k] = Jx * By - Jy * Bx;
}

// -------------------------------------------------------------------------------------------
// Fluid single-step predictor (Sec. 3.3, Sec. 5.1):
//   rho' = sum_i [1.5 f_i(x - e_i) - f_i(x) + 0.5 f_i(x + e_i)]
//   rho' u* = sum_i e_i {f_i(x - e_i) + (tau - 1)[f_i(x + e_i) - 2 f_i(x) + f_i(x - e_i)]}
//             - (tau/2) sum_i e_i [F_i(x + e_i) - F_i(x - e_i)] + F(x)
// with f_i = f_i^eq(rho, u) and F_i = (1 - 1/(2 tau)) w_i [3 (e_i - u) . F + 9 (e_i . u)(e_i . F)].
//
// Evaluated as an increment per pair of opposite neighbours y+ = x + d, y- = x - d (weight w).
// Writing f_i = w_i + h_i, h_i = w_i [drho + (1 + drho) q_i], q_i = 3 e.u + q2, q2 =
// 4.5 (e.u)^2 - 1.5 u.u, J = (1 + drho) u, the parts that do not depend on the neighbours
// cancel analytically (sum_i w_i = 1, sum_i w_i q_i = 0, sum_i w_i e_i e_i = I/3) and
//   drho' - drho = sum_pairs w [2 (Ddrho+ + Ddrho-) + 2 (DQ+ + DQ-) + 3 d.(J- - J+)]
//   rho' u* - rho u = sum_pairs d w [(drho- - drho+) + 3 (2 tau - 1) d.(DJ- + DJ+) + (DQ- - DQ+)]
//                     - tau c_F sum_pairs d w (G+ - G-) + F(x)
// with D. = value at y+- minus value at x (DQ compares (1 + drho) q2 along the same d),
// G = 9 (d.u)(d.F) - 3 u.F and c_F = 1 - 1/(2 tau). Every term is a neighbour difference, so the
// float32 rounding is relative to the change of the step, and the new state is
// drho' = drho + delta, u* = u + (Dm - delta u) / (1 + drho').
// -------------------------------------------------------------------------------------------
__constant__ int c_pair[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0},
                                 {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};

template <typename TR, typename TU, bool BATCH>
__global__ void __launch_bounds__(kCellThreads) k_fluid(const TR *rho, const TU *u, const float *F, TR *rho_o,
                                                        TU *u_o, StepConst c, const PipeStep *tab,
                                                        const BlockMap *map) {
    int64_t blk = blockIdx.x;
    if constexpr (BATCH) {
        const BlockMap m = map[blk];
        const PipeStep &q = tab[m.pipe];
        rho = (const TR *)q.rho;
        u = (const TU *)q.u;
        F = q.F;
        rho_o = (TR *)q.rho_o;
        u_o = (TU *)q.u_o;
        c = q.c;
        blk = m.local;
    }
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    const int64_t k = blk * kCellThreads + threadIdx.x;
    if (k >= N) return;
    const int x = (int)(k % c.nx);
    const int y = (int)((k / c.nx) % c.ny);
    const int z = (int)(k / ((int64_t)c.nx * c.ny));
    const float tau = c.tau, us = c.u_scale;
    const float cF = 1.0f - 0.5f / tau;
    const float a3 = 3.0f * (2.0f * tau - 1.0f);

    const float d0 = St<TR>::ld(rho, k);
    const float ux0 = St<TU>::ld(u, k) * us, uy0 = St<TU>::ld(u, N + k) * us, uz0 = St<TU>::ld(u, 2 * N + k) * us;
    const float uu0 = ux0 * ux0 + uy0 * uy0 + uz0 * uz0;
    float dr = 0.f;
    float m0 = 0.f, m1 = 0.f, m2 = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const int ex = c_pair[i][0], ey = c_pair[i][1], ez = c_pair[i][2];
        const float w = i < 3 ? WF : WE;
        const int64_t kp = wrapi(x + ex, c.nx) + (int64_t)c.nx * (wrapi(y + ey, c.ny) + (int64_t)c.ny * wrapi(z + ez, c.nz));
        const int64_t km = wrapi(x - ex, c.nx) + (int64_t)c.nx * (wrapi(y - ey, c.ny) + (int64_t)c.ny * wrapi(z - ez, c.nz));
        const float dp = St<TR>::ld(rho, kp), dm = St<TR>::ld(rho, km);
        const float upx = St<TU>::ld(u, kp) * us, upy = St<TU>::ld(u, N + kp) * us, upz = St<TU>::ld(u, 2 * N + kp) * us;
        const float umx = St<TU>::ld(u, km) * us, umy = St<TU>::ld(u, N + km) * us, umz = St<TU>::ld(u, 2 * N + km) * us;
        const float fpx = F[kp], fpy = F[N + kp], fpz = F[2 * N + kp];
        const float fmx = F[km], fmy = F[N + km], fmz = F[2 * N + km];
        // differences to the centre
        const float Dpx = upx - ux0, Dpy = upy - uy0, Dpz = upz - uz0;
        const float Dmx = umx - ux0, Dmy = umy - uy0, Dmz = umz - uz0;
        const float Ddp = dp - d0, Ddm = dm - d0;
        const float eu0 = ex * ux0 + ey * uy0 + ez * uz0;
        const float eDp = ex * Dpx + ey * Dpy + ez * Dpz, eDm = ex * Dmx + ey * Dmy + ez * Dmz;
        const float eup = eu0 + eDp, eum = eu0 + eDm;
        // (1 + drho) q2 differences along d: q2(u+-) - q2(u0) = 4.5 (d.D)(d.S) - 1.5 D.S, S = u+- + u0
        const float q20 = 4.5f * eu0 * eu0 - 1.5f * uu0;
        const float dq2p = 4.5f * eDp * (eup + eu0) - 1.5f * (Dpx * (upx + ux0) + Dpy * (upy + uy0) + Dpz * (upz + uz0));
        const float dq2m = 4.5f * eDm * (eum + eu0) - 1.5f * (Dmx * (umx + ux0) + Dmy * (umy + uy0) + Dmz * (umz + uz0));
        const float DQp = (1.0f + dp) * dq2p + Ddp * q20, DQm = (1.0f + dm) * dq2m + Ddm * q20;
        // momentum differences along d: d.(J+- - J0) = d.D + (drho+- d.u+- - drho0 d.u0)
        const float dJp = eDp + (dp * eup - d0 * eu0), dJm = eDm + (dm * eum - d0 * eu0);
        dr += w * (2.0f * (Ddp + Ddm) + 2.0f * (DQp + DQm) + 3.0f * (dJm - dJp));
        const float cm = w * ((dm - dp) + a3 * (dJm + dJp) + (DQm - DQp));
        m0 += ex * cm;
        m1 += ey * cm;
        m2 += ez * cm;
        const float efp = ex * fpx + ey * fpy + ez * fpz, efm = ex * fmx + ey * fmy + ez * fmz;
        const float Gp = 9.0f * eup * efp - 3.0f * (upx * fpx + upy * fpy + upz * fpz);
        const float Gm = 9.0f * eum * efm - 3.0f * (umx * fmx + umy * fmy + umz * fmz);
        const float cg = w * (Gp - Gm);
        g0 += ex * cg;
        g1 += ey * cg;
        g2 += ez * cg;
    }
    const float dnew = d0 + dr;
    const float tcF = tau * cF;
    const float Dm0 = (m0 - tcF * g0) + F[k];
    const float Dm1 = (m1 - tcF * g1) + F[N + k];
    const float Dm2 = (m2 - tcF * g2) + F[2 * N + k];
    const float inv = 1.0f / (1.0f + dnew);
    St<TR>::st(rho_o, k, dnew);
    St<TU>::st(u_o, k, (ux0 + (Dm0 - dr * ux0) * inv) * c.inv_u_scale);
    St<TU>::st(u_o, N + k, (uy0 + (Dm1 - dr * uy0) * inv) * c.inv_u_scale);
    St<TU>::st(u_o, 2 * N + k, (uz0 + (Dm2 - dr * uz0) * inv) * c.inv_u_scale);
}

// -------------------------------------------------------------------------------------------
// Float64 reductions with a fixed summation order: a fixed grid of kRedBlocks workgroups walks
// the cells with a fixed stride, each block tree-reduces in LDS and writes one partial; a
// single block then sums the partials in index order.
// -------------------------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_sum(double (*sh)[kRedThreads], double *v) {
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int q = 0; q < NV; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + w];
        }
        __syncthreads();
    }
}

template <typename TU, bool BATCH>
__global__ void __launch_bounds__(kRedThreads) k_flow_partial(const TU *u, double *part, StepConst c,
                                                              const PipeStep *tab) {
    int blk = blockIdx.x;
    if constexpr (BATCH) {  // kRedBlocks workgroups per box
        const PipeStep &q = tab[blockIdx.x / kRedBlocks];
        if (!q.c.flow_control) return;
        u = (const TU *)q.u_o;
        part = q.flow_part;
        c = q.c;
        blk = blockIdx.x % kRedBlocks;
    }
    __shared__ double sh[1][kRedThreads];
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    const double R2 = c.radius * c.radius;
    double s = 0.0;
    for (int64_t k = (int64_t)blk * kRedThreads + threadIdx.x; k < N; k += (int64_t)kRedBlocks * kRedThreads) {
        const int y = (int)((k / c.nx) % c.ny);
        const int z = (int)(k / ((int64_t)c.nx * c.ny));
        const double dy = y - c.yc, dz = z - c.zc;
        if (dy * dy + dz * dz <= R2) s += (double)(St<TU>::ld(u, k) * c.u_scale);
    }
    double v[1] = {s};
    block_sum<1>(sh, v);
    if (threadIdx.x == 0) part[blk] = sh[0][0];
}

// partial layout: 0 Ek, 1 Em, 2 Eb, 3 sum u_x (Omega), 4 Pp, 5 Pnu/nu, 6 PL, 7 Meta/eta, 8 Madv,
// 9 sum |J|^2, 10 mass, 11 Q sum, 12 n_omega, 13 max |u|^2, 14 nonfinite, 15 unused
template <typename TR, typename TU, typename TB>
__global__ void __launch_bounds__(kRedThreads) k_budget_partial(const TR *rho, const TU *u, const TB *b,
                                                                const float *bext, double *part, StepConst c) {
    __shared__ double sh[13][kRedThreads];
    __shared__ double shm[kRedThreads];
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    const double us = c.u_scale, bs = c.b_scale;
    const double R2 = c.radius * c.radius;
    const double Ro = c.radius - 2.0, Ro2 = Ro * Ro;
    double v[13];
#pragma unroll
    for (int q = 0; q < 13; ++q) v[q] = 0.0;
    double umax2 = 0.0;
    double nonfin = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; k < N; k += (int64_t)kRedBlocks * kRedThreads) {
        const int x = (int)(k % c.nx);
        const int y = (int)((k / c.nx) % c.ny);
        const int z = (int)(k / ((int64_t)c.nx * c.ny));
        const double r = 1.0 + (double)St<TR>::ld(rho, k);
        double uu[3], bb[3], B[3];
        for (int a = 0; a < 3; ++a) {
            uu[a] = (double)St<TU>::ld(u, a * N + k) * us;
            bb[a] = (double)St<TB>::ld(b, a * N + k) * bs;
            B[a] = bb[a] + (double)bext[a * c.nx + x];
        }
        const double u2 = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
        if (!isfinite(u2) || !isfinite(r)) nonfin = 1.0;
        umax2 = fmax(umax2, u2);
        v[10] += r;
        const double dy = y - c.yc, dz = z - c.zc, r2 = dy * dy + dz * dz;
        if (r2 <= R2) v[11] += uu[0];
        if (r2 >= Ro2) continue;
        v[12] += 1.0;
        double grho[3] = {0, 0, 0}, lu[3] = {0, 0, 0}, lb[3] = {0, 0, 0}, divL[3] = {0, 0, 0};
        double gb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int i = 0; i < 18; ++i) {
            const int e[3] = {c_dir[i][0], c_dir[i][1], c_dir[i][2]};
            const double w = i < 6 ? 1.0 / 18.0 : 1.0 / 36.0;
            const int xn = wrapi(x + e[0], c.nx);
            const int64_t kn = xn + (int64_t)c.nx * (wrapi(y + e[1], c.ny) + (int64_t)c.ny * wrapi(z + e[2], c.nz));
            const double rn = 1.0 + (double)St<TR>::ld(rho, kn);
            double un[3], bn[3], Bn[3];
            for (int a = 0; a < 3; ++a) {
                un[a] = (double)St<TU>::ld(u, a * N + kn) * us;
                bn[a] = (double)St<TB>::ld(b, a * N + kn) * bs;
                Bn[a] = bn[a] + (double)bext[a * c.nx + xn];
            }
            for (int a = 0; a < 3; ++a) {
                grho[a] += 3.0 * w * e[a] * rn;
                lu[a] += 6.0 * w * (un[a] - uu[a]);
                lb[a] += 6.0 * w * (bn[a] - bb[a]);
                double dl = 0.0;
                for (int cc = 0; cc < 3; ++cc) {
                    gb[a][cc] += 3.0 * w * e[cc] * bn[a];
                    dl += e[cc] * (un[cc] * Bn[a] - Bn[cc] * un[a]);
                }
                divL[a] += 3.0 * w * dl;
            }
        }
        const double J[3] = {gb[2][1] - gb[1][2], gb[0][2] - gb[2][0], gb[1][0] - gb[0][1]};
        const double JxB[3] = {J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2], J[0] * B[1] - J[1] * B[0]};
        v[0] += 0.5 * r * u2;
        v[1] += 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
        v[2] += 0.5 * (bb[0] * bb[0] + bb[1] * bb[1] + bb[2] * bb[2]);
        v[3] += uu[0];
        for (int a = 0; a < 3; ++a) {
            v[4] += -uu[a] * (grho[a] / 3.0);
            v[5] += uu[a] * lu[a];
            v[6] += uu[a] * JxB[a];
            v[7] += B[a] * lb[a];
            v[8] += -B[a] * divL[a];
            v[9] += J[a] * J[a];
        }
    }
    block_sum<13>(sh, v);
    // max |u|^2 and "any non-finite" in the same fixed tree
    __shared__ double shf[kRedThreads];
    shm[threadIdx.x] = umax2;
    shf[threadIdx.x] = nonfin;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + w]);
            shf[threadIdx.x] = fmax(shf[threadIdx.x], shf[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *o = part + (int64_t)blockIdx.x * kBudgetVals;
        for (int q = 0; q < 13; ++q) o[q] = sh[q][0];
        o[13] = shm[0];
        o[14] = shf[0];
        o[15] = 0.0;
    }
}

__global__ void __launch_bounds__(kRedThreads) k_budget_final(const double *part, DevCtrl *ctrl, mhd_budget *ring,
                                                              StepConst c) {
    __shared__ double sh[13][kRedThreads];
    __shared__ double shm[kRedThreads], shf[kRedThreads];
    double v[13];
#pragma unroll
    for (int q = 0; q < 13; ++q) v[q] = 0.0;
    double m = 0.0, f = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) {
        const double *p = part + (int64_t)i * kBudgetVals;
#pragma unroll
        for (int q = 0; q < 13; ++q) v[q] += p[q];
        m = fmax(m, p[13]);
        f = fmax(f, p[14]);
    }
    block_sum<13>(sh, v);
    shm[threadIdx.x] = m;
    shf[threadIdx.x] = f;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            shm[threadIdx.x] = fmax(shm[threadIdx.x], shm[threadIdx.x + w]);
            shf[threadIdx.x] = fmax(shf[threadIdx.x], shf[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = sh[12][0];
        const double inv = n > 0.0 ? 1.0 / n : 0.0;
        mhd_budget r;
        r.step = ctrl->t;
        r.G = ctrl->G_step;
        r.E_k = sh[0][0] * inv;
        r.E_m = sh[1][0] * inv;
        r.E_b = sh[2][0] * inv;
        r.P_in = r.G * sh[3][0] * inv;
        r.P_p = sh[4][0] * inv;
        r.P_nu = c.nu * sh[5][0] * inv;
        r.P_L = sh[6][0] * inv;
        r.M_eta = c.eta * sh[7][0] * inv;
        r.M_adv = sh[8][0] * inv;
        r.joule = c.eta * sh[9][0] * inv;
        r.mass = sh[10][0];
        r.Q = sh[11][0] / (double)c.nx;
        r.u_max = sqrt(shm[0]);
        r.n_omega = n;
        // |u| >= c_s = 1/sqrt(3) or a non-finite value marks the run unstable
        if (shf[0] != 0.0 || !(shm[0] < 1.0 / 3.0) || !isfinite(sh[0][0])) ctrl->status |= 1;
        const int idx = ctrl->n_records;
        if (idx < kRingCap) {
            ring[idx] = r;
            ctrl->n_records = idx + 1;
        } else {
            ctrl->overflow += 1;
        }
    }
}

// -------------------------------------------------------------------------------------------
// Storage conversion (float32 staging <-> storage kind)
// -------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_store(const float *src, T *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        St<T>::st(dst, i, src[i]);
}
template <typename T>
__global__ void k_load(const T *src, float *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = St<T>::ld(src, i);
}

// ===========================================================================================
// Host-side launch wrappers
// ===========================================================================================
static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_ctrl_begin(hipStream_t s, DevCtrl *ctrl, StepConst c) {
    hipLaunchKernelGGL(k_ctrl_begin, dim3(1), dim3(64), 0, s, ctrl, c);
    return hipGetLastError();
}

hipError_t launch_step_end(hipStream_t s, DevCtrl *ctrl, const double *flow_part, StepConst c, double inv_count) {
    hipLaunchKernelGGL(k_step_end<false>, dim3(1), dim3(kRedThreads), 0, s, ctrl, flow_part, c, inv_count, nullptr);
    return hipGetLastError();
}

hipError_t launch_ctrl_begin_batch(hipStream_t s, const PipeStep *tab, int n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ctrl_begin_batch, dim3(n), dim3(64), 0, s, tab);
    return hipGetLastError();
}

hipError_t launch_step_end_batch(hipStream_t s, const PipeStep *tab, int n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_step_end<true>, dim3(n), dim3(kRedThreads), 0, s, nullptr, nullptr, StepConst{}, 0.0, tab);
    return hipGetLastError();
}

hipError_t launch_reset_records(hipStream_t s, DevCtrl *ctrl) {
    hipLaunchKernelGGL(k_reset_records, dim3(1), dim3(64), 0, s, ctrl);
    return hipGetLastError();
}

SweepArgs make_sweep_args(const void *u, const void *b, void *bo, const float *bext, StepConst c, SweepLaunch L) {
    SweepArgs a;
    a.u = u;
    a.b = b;
    a.bo = bo;
    a.bext = bext;
    a.nx = c.nx;
    a.ny = c.ny;
    a.nz = c.nz;
    const bool pair = L.pair && c.nx % 128 == 0;
    const int tx = pair ? 128 : L.tx;
    const int ty = pair ? (L.ty >= 8 ? 8 : 4) : 256 / L.tx;
    a.tiles_x = (c.nx + tx - 1) / tx;
    a.tiles_y = (c.ny + ty - 1) / ty;
    a.zchunk = L.zchunk;
    a.nzc = (c.nz + L.zchunk - 1) / L.zchunk;
    a.nblocks = a.tiles_x * a.tiles_y * a.nzc;
    a.kappa = c.kappa;
    a.u_scale = c.u_scale;
    a.b_scale = c.b_scale;
    a.inv_b_scale = c.inv_b_scale;
    return a;
}

// grid of a sweep launch: a multiple of 8 so the XCD-aware remap is a permutation
static inline unsigned sweep_grid(int nblocks) { return (unsigned)(((nblocks + 7) / 8) * 8); }

template <typename TU, typename TB, bool BATCH>
static hipError_t sweep_typed(hipStream_t s, const SweepArgs &a, SweepLaunch L, const PipeStep *tab,
                              const BlockMap *map, int parity, int nblocks) {
    const dim3 grid(sweep_grid(nblocks));
    if (L.pair) {
        if (L.ty >= 8)
            hipLaunchKernelGGL((k_mag_sweep_pair<8, TU, TB, BATCH>), grid, dim3(512), 0, s, a, tab, map, parity, nblocks);
        else
            hipLaunchKernelGGL((k_mag_sweep_pair<4, TU, TB, BATCH>), grid, dim3(256), 0, s, a, tab, map, parity, nblocks);
        return hipGetLastError();
    }
    switch (L.tx) {
        case 64:
            hipLaunchKernelGGL((k_mag_sweep<64, 4, TU, TB, BATCH>), grid, dim3(256), 0, s, a, tab, map, parity, nblocks);
            break;
        case 32:
            hipLaunchKernelGGL((k_mag_sweep<32, 8, TU, TB, BATCH>), grid, dim3(256), 0, s, a, tab, map, parity, nblocks);
            break;
        case 16:
            hipLaunchKernelGGL((k_mag_sweep<16, 16, TU, TB, BATCH>), grid, dim3(256), 0, s, a, tab, map, parity, nblocks);
            break;
        default:
            hipLaunchKernelGGL((k_mag_sweep<8, 32, TU, TB, BATCH>), grid, dim3(256), 0, s, a, tab, map, parity, nblocks);
            break;
    }
    return hipGetLastError();
}

// Supported storage mixes: all float32; rho f16 with u f16 or bf16 and b f16; all bf16.
#define MHD_KIND_F32 0
#define MHD_KIND_F16 1
#define MHD_KIND_BF16 2

template <bool BATCH>
static hipError_t sweep_kinds(hipStream_t s, int kinds, const SweepArgs &a, SweepLaunch L, const PipeStep *tab,
                              const BlockMap *map, int parity, int nblocks) {
    const int ku = (kinds >> 4) & 15, kb = (kinds >> 8) & 15;
    if (ku == MHD_KIND_F32 && kb == MHD_KIND_F32)
        return sweep_typed<float, float, BATCH>(s, a, L, tab, map, parity, nblocks);
    if (ku == MHD_KIND_F16 && kb == MHD_KIND_F16)
        return sweep_typed<__half, __half, BATCH>(s, a, L, tab, map, parity, nblocks);
    if (ku == MHD_KIND_BF16 && kb == MHD_KIND_F16)
        return sweep_typed<__hip_bfloat16, __half, BATCH>(s, a, L, tab, map, parity, nblocks);
    if (ku == MHD_KIND_BF16 && kb == MHD_KIND_BF16)
        return sweep_typed<__hip_bfloat16, __hip_bfloat16, BATCH>(s, a, L, tab, map, parity, nblocks);
    return hipErrorInvalidValue;
}

hipError_t launch_mag_sweep(hipStream_t s, int kinds, const void *u, const void *b, void *bo, const float *bext,
                            StepConst c, SweepLaunch L) {
    L.pair = L.pair && c.nx % 128 == 0;
    const SweepArgs a = make_sweep_args(u, b, bo, bext, c, L);
    return sweep_kinds<false>(s, kinds, a, L, nullptr, nullptr, 0, a.nblocks);
}

hipError_t launch_mag_sweep_batch(hipStream_t s, int kinds, SweepLaunch L, const PipeStep *tab, const BlockMap *map,
                                  int parity, int nblocks) {
    if (nblocks <= 0) return hipSuccess;
    return sweep_kinds<true>(s, kinds, SweepArgs{}, L, tab, map, parity, nblocks);
}

#define MHD_DISPATCH1(kind, FN, ...)                                       \
    switch (kind) {                                                        \
        case MHD_KIND_F32: return FN<float>(__VA_ARGS__);                  \
        case MHD_KIND_F16: return FN<__half>(__VA_ARGS__);                 \
        case MHD_KIND_BF16: return FN<__hip_bfloat16>(__VA_ARGS__);        \
        default: return hipErrorInvalidValue;                              \
    }

template <typename T>
static hipError_t ib_t(hipStream_t s, void *phi, float scale, float inv_scale, const IbArgs &a) {
    if (a.M <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ib_interp<T, false>), dim3(blocks_for(a.M, kIbThreads)), dim3(kIbThreads), 0, s,
                       (const T *)phi, scale, a, nullptr, nullptr, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.nband <= 0) return e;
    hipLaunchKernelGGL((k_ib_spread<T, false>), dim3(blocks_for(a.nband, kIbThreads)), dim3(kIbThreads), 0, s,
                       (T *)phi, scale, inv_scale, a, nullptr, nullptr, 0);
    return hipGetLastError();
}
hipError_t launch_ib(hipStream_t s, int kind, void *phi, float scale, float inv_scale, const IbArgs &a) {
    MHD_DISPATCH1(kind, ib_t, s, phi, scale, inv_scale, a)
}

template <typename T>
static hipError_t ib_interp_batch_t(hipStream_t s, const PipeStep *tab, const BlockMap *map, int which, int nblocks) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ib_interp<T, true>), dim3(nblocks), dim3(kIbThreads), 0, s, nullptr, 0.f, IbArgs{}, tab, map,
                       which);
    return hipGetLastError();
}
hipError_t launch_ib_interp_batch(hipStream_t s, int kind, const PipeStep *tab, const BlockMap *map, int which,
                                  int nblocks) {
    MHD_DISPATCH1(kind, ib_interp_batch_t, s, tab, map, which, nblocks)
}
template <typename T>
static hipError_t ib_spread_batch_t(hipStream_t s, const PipeStep *tab, const BlockMap *map, int which, int nblocks) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_ib_spread<T, true>), dim3(nblocks), dim3(kIbThreads), 0, s, nullptr, 0.f, 0.f, IbArgs{}, tab,
                       map, which);
    return hipGetLastError();
}
hipError_t launch_ib_spread_batch(hipStream_t s, int kind, const PipeStep *tab, const BlockMap *map, int which,
                                  int nblocks) {
    MHD_DISPATCH1(kind, ib_spread_batch_t, s, tab, map, which, nblocks)
}

template <typename T>
static hipError_t lorentz_t(hipStream_t s, const void *b, const float *bext, const DevCtrl *ctrl, float *F,
                            StepConst c) {
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    hipLaunchKernelGGL((k_lorentz<T, false>), dim3(blocks_for(N, kCellThreads)), dim3(kCellThreads), 0, s,
                       (const T *)b, c.b_scale, bext, ctrl, F, c, nullptr, nullptr);
    return hipGetLastError();
}
hipError_t launch_lorentz(hipStream_t s, int kind_b, const void *b, const float *bext, const DevCtrl *ctrl, float *F,
                          StepConst c) {
    MHD_DISPATCH1(kind_b, lorentz_t, s, b, bext, ctrl, F, c)
}
template <typename T>
static hipError_t lorentz_batch_t(hipStream_t s, const PipeStep *tab, const BlockMap *map, int nblocks) {
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_lorentz<T, true>), dim3(nblocks), dim3(kCellThreads), 0, s, nullptr, 0.f, nullptr, nullptr,
                       nullptr, StepConst{}, tab, map);
    return hipGetLastError();
}
hipError_t launch_lorentz_batch(hipStream_t s, int kind_b, const PipeStep *tab, const BlockMap *map, int nblocks) {
    MHD_DISPATCH1(kind_b, lorentz_batch_t, s, tab, map, nblocks)
}

template <typename TR, typename TU, bool BATCH>
static hipError_t fluid_t(hipStream_t s, const void *rho, const void *u, const float *F, void *rho_o, void *u_o,
                          StepConst c, const PipeStep *tab, const BlockMap *map, int nblocks) {
    if (!BATCH) nblocks = (int)blocks_for((int64_t)c.nx * c.ny * c.nz, kCellThreads);
    if (nblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_fluid<TR, TU, BATCH>), dim3(nblocks), dim3(kCellThreads), 0, s, (const TR *)rho,
                       (const TU *)u, F, (TR *)rho_o, (TU *)u_o, c, tab, map);
    return hipGetLastError();
}
template <bool BATCH>
static hipError_t fluid_kinds(hipStream_t s, int kinds, const void *rho, const void *u, const float *F, void *rho_o,
                              void *u_o, StepConst c, const PipeStep *tab, const BlockMap *map, int nblocks) {
    const int kr = kinds & 15, ku = (kinds >> 4) & 15;
    if (kr == MHD_KIND_F32 && ku == MHD_KIND_F32)
        return fluid_t<float, float, BATCH>(s, rho, u, F, rho_o, u_o, c, tab, map, nblocks);
    if (kr == MHD_KIND_F16 && ku == MHD_KIND_F16)
        return fluid_t<__half, __half, BATCH>(s, rho, u, F, rho_o, u_o, c, tab, map, nblocks);
    if (kr == MHD_KIND_F16 && ku == MHD_KIND_BF16)
        return fluid_t<__half, __hip_bfloat16, BATCH>(s, rho, u, F, rho_o, u_o, c, tab, map, nblocks);
    if (kr == MHD_KIND_BF16 && ku == MHD_KIND_BF16)
        return fluid_t<__hip_bfloat16, __hip_bfloat16, BATCH>(s, rho, u, F, rho_o, u_o, c, tab, map, nblocks);
    return hipErrorInvalidValue;
}
hipError_t launch_fluid(hipStream_t s, int kinds, const void *rho, const void *u, const float *F, void *rho_o,
                        void *u_o, StepConst c) {
    return fluid_kinds<false>(s, kinds, rho, u, F, rho_o, u_o, c, nullptr, nullptr, 0);
}
hipError_t launch_fluid_batch(hipStream_t s, int kinds, const PipeStep *tab, const BlockMap *map, int nblocks) {
    return fluid_kinds<true>(s, kinds, nullptr, nullptr, nullptr, nullptr, nullptr, StepConst{}, tab, map, nblocks);
}

template <typename T>
static hipError_t flow_t(hipStream_t s, const void *u, double *part, StepConst c) {
    hipLaunchKernelGGL((k_flow_partial<T, false>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, (const T *)u, part, c,
                       nullptr);
    return hipGetLastError();
}
hipError_t launch_flow_partial(hipStream_t s, int kind_u, const void *u, double *part, StepConst c) {
    MHD_DISPATCH1(kind_u, flow_t, s, u, part, c)
}
template <typename T>
static hipError_t flow_batch_t(hipStream_t s, const PipeStep *tab, int n) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_flow_partial<T, true>), dim3(n * kRedBlocks), dim3(kRedThreads), 0, s, nullptr, nullptr,
                       StepConst{}, tab);
    return hipGetLastError();
}
hipError_t launch_flow_partial_batch(hipStream_t s, int kind_u, const PipeStep *tab, int n) {
    MHD_DISPATCH1(kind_u, flow_batch_t, s, tab, n)
}

template <typename TR, typename TU, typename TB>
static hipError_t budget_t(hipStream_t s, const void *rho, const void *u, const void *b, const float *bext,
                           DevCtrl *ctrl, double *part, mhd_budget *ring, StepConst c) {
    hipLaunchKernelGGL((k_budget_partial<TR, TU, TB>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, (const TR *)rho,
                       (const TU *)u, (const TB *)b, bext, part, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_budget_final, dim3(1), dim3(kRedThreads), 0, s, part, ctrl, ring, c);
    return hipGetLastError();
}
hipError_t launch_budget(hipStream_t s, int kinds, const void *rho, const void *u, const void *b, const float *bext,
                         DevCtrl *ctrl, double *part, mhd_budget *ring, StepConst c) {
    const int kr = kinds & 15, ku = (kinds >> 4) & 15, kb = (kinds >> 8) & 15;
    if (kr == MHD_KIND_F32 && ku == MHD_KIND_F32 && kb == MHD_KIND_F32)
        return budget_t<float, float, float>(s, rho, u, b, bext, ctrl, part, ring, c);
    if (kr == MHD_KIND_F16 && ku == MHD_KIND_F16 && kb == MHD_KIND_F16)
        return budget_t<__half, __half, __half>(s, rho, u, b, bext, ctrl, part, ring, c);
    if (kr == MHD_KIND_F16 && ku == MHD_KIND_BF16 && kb == MHD_KIND_F16)
        return budget_t<__half, __hip_bfloat16, __half>(s, rho, u, b, bext, ctrl, part, ring, c);
    if (kr == MHD_KIND_BF16 && ku == MHD_KIND_BF16 && kb == MHD_KIND_BF16)
        return budget_t<__hip_bfloat16, __hip_bfloat16, __hip_bfloat16>(s, rho, u, b, bext, ctrl, part, ring, c);
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t store_t(hipStream_t s, const float *src, void *dst, int64_t n) {
    hipLaunchKernelGGL(k_store<T>, dim3((unsigned)std::min<int64_t>(blocks_for(n, 256), 65536)), dim3(256), 0, s, src,
                       (T *)dst, n);
    return hipGetLastError();
}
hipError_t launch_store_kind(hipStream_t s, int kind, const float *src, void *dst, int64_t n) {
    MHD_DISPATCH1(kind, store_t, s, src, dst, n)
}

template <typename T>
static hipError_t load_t(hipStream_t s, const void *src, float *dst, int64_t n) {
    hipLaunchKernelGGL(k_load<T>, dim3((unsigned)std::min<int64_t>(blocks_for(n, 256), 65536)), dim3(256), 0, s,
                       (const T *)src, dst, n);
    return hipGetLastError();
}
hipError_t launch_load_kind(hipStream_t s, int kind, const void *src, float *dst, int64_t n) {
    MHD_DISPATCH1(kind, load_t, s, src, dst, n)
}

}  // namespace mhd
