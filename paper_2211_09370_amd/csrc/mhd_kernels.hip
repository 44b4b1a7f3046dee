// gfx950 kernels of the single-step simplified lattice Boltzmann step for quasi-static MHD pipe
// flow (arXiv:2211.09370). All arithmetic is float32 except the budget / flow-rate reductions,
// which convert the stored values to float64 and sum them in a fixed order.
//
// Field layout: component-major, x fastest; element (a, x, y, z) at a*N + x + nx*(y + ny*z).
// Storage kinds: float32, or 16-bit offsets (rho - 1 in every kind, u / u_scale, b / b_scale).
//
// Kernels (per fluid step, in order):
//   k_ctrl_begin   body force G(t) of the step (Sec. 4, variable-force form)
//   k_mag_sweep    x n_mag: b*(x) = sum_i g_i^eq(x - e_i), tau_m = 1, c = 6 eta (Sec. 5.7);
//                  in mhd_sweep.hip
//   k_ib_interp    per marker: delta_j = s_j (b_wall - sum_k D_jk phi_k)     (Sec. 5.4 / 5.6)
//   k_ib_spread    per wall-band cell: phi_k += sum_j D_jk delta_j (gather form, no atomics)
//   k_lorentz      F = G x + (curl b) x (B_ext + b), isotropic differences    (Sec. 5.1)
//   k_fluid        single-step rho, rho u with GZS forcing + discrete-effect term (Sec. 3.3, 5.1),
//                  rescaled by gamma (Sec. 7); macroscopic tau = 1 update for tau >= 1 (Sec. 5.7)
//   k_ib_interp / k_ib_spread on u                                              (Sec. 5.3 / 5.5)
//   k_flow_partial + k_step_end   flow-rate control sum (float64), step counter
//   k_budget_partial + k_budget_final   every K steps: energy budgets of Sec. 4 (float64)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mhd_device.h"

namespace mhd {

// Neighbour offsets without the rest direction: 6 faces, 12 edges (the D3Q19 set), then the 8
// corners of D3Q27. Weights: D3Q19 faces 1/18, edges 1/36; D3Q27 faces 2/27, edges 1/54,
// corners 1/216.
__constant__ int c_dir[26][3] = {{1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                                 {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1},
                                 {1, 0, -1}, {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
                                 {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1},
                                 {-1, 1, 1}, {1, -1, -1}};
// The same offsets as compile-time values, for the fully unrolled loops of the cell updates (the
// offsets then become immediates instead of scalar loads kept live across a plane march).
__device__ constexpr int dir_of(int i, int a) {
    constexpr int t[26][3] = {{1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                              {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1},
                              {1, 0, -1}, {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
                              {1, 1, 1},  {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1},
                              {-1, 1, 1}, {1, -1, -1}};
    return t[i][a];
}
// weight of neighbour i of c_dir on either lattice
__device__ __forceinline__ float dir_weight(int i, bool q27) {
    if (q27) return i < 6 ? 2.0f / 27.0f : i < 18 ? 1.0f / 54.0f : 1.0f / 216.0f;
    return i < 6 ? WF : WE;
}
__device__ __forceinline__ double dir_weight_d(int i, bool q27) {
    if (q27) return i < 6 ? 2.0 / 27.0 : i < 18 ? 1.0 / 54.0 : 1.0 / 216.0;
    return i < 6 ? 1.0 / 18.0 : 1.0 / 36.0;
}

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

// Sums and maxima over a wave with cross-lane shuffles in a fixed butterfly (every lane ends
// with the same bits), then over the workgroup's waves through LDS in wave order: the result is
// the same on every run. Results are valid in thread 0.
constexpr int kRedWaves = kRedThreads / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
// NV sums and NM maxima of the workgroup, in place in thread 0's v and m
template <int NV, int NM>
__device__ __forceinline__ void block_reduce(double (*sh)[kRedWaves], double *v, double *m) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
#pragma unroll
    for (int q = 0; q < NM; ++q) m[q] = wave_max(m[q]);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) sh[q][wv] = v[q];
#pragma unroll
        for (int q = 0; q < NM; ++q) sh[NV + q][wv] = m[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            double t = sh[q][0];
            for (int i = 1; i < kRedWaves; ++i) t += sh[q][i];
            v[q] = t;
        }
#pragma unroll
        for (int q = 0; q < NM; ++q) {
            double t = sh[NV + q][0];
            for (int i = 1; i < kRedWaves; ++i) t = fmax(t, sh[NV + q][i]);
            m[q] = t;
        }
    }
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
    __shared__ double sh[1][kRedWaves];
    double s[1] = {0.0};
    if (c.flow_control)
        for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) s[0] += part[i];
    block_reduce<1, 0>(sh, s, nullptr);
    if (threadIdx.x == 0) {
        if (c.flow_control) {
            double ub = s[0] * inv_count;
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
// Where the taps of a marker and the gather entries of a band cell come from: the general
// padded structure-of-arrays tables, or (line-structured walls) the tables of the marker's line
// and of the cell's band row, whose wave-uniform index lets them be read with scalar loads.
// Both list taps and entries in the same order, so the two forms give the same bits.
struct GeneralTaps {
    const int *cell;
    const float *w;
    int64_t M;
    int j;
    __device__ int64_t k(int t) const { return cell[(int64_t)t * M + j]; }
    __device__ float wt(int t) const { return w[(int64_t)t * M + j]; }
};
struct LineTaps {
    const int *off;  // this line's tap offsets
    const float *w;
    int x;
    __device__ int64_t k(int t) const { return x + off[t]; }
    __device__ float wt(int t) const { return w[t]; }
};
struct GeneralEntries {
    const int *mk;
    const float *w;
    int nband, e;
    __device__ int j(int q) const { return mk[(int64_t)q * nband + e]; }
    __device__ float wt(int q) const { return w[(int64_t)q * nband + e]; }
};
struct RowEntries {
    const int *mk;  // this row's entry lines
    const float *w;
    int nx, x;
    __device__ int j(int q) const { return mk[q] * nx + x; }
    __device__ float wt(int q) const { return w[q]; }
};

template <typename T, typename Taps>
__device__ __forceinline__ void ib_marker(const T *phi, float scale, const IbArgs &a, int j, const Taps &tp,
                                          float &d0, float &d1, float &d2) {
    float I0 = 0.f, I1 = 0.f, I2 = 0.f;
    const T *hi = (const T *)a.phi_hi;
    if (hi) {  // split form: the field is (hi + lo) scale
#pragma unroll 9
        for (int t = 0; t < a.tm; ++t) {
            const int64_t k = tp.k(t);
            const float w = tp.wt(t);
            I0 += w * ((St<T>::ld(phi, k) + St<T>::ld(hi, k)) * scale);
            I1 += w * ((St<T>::ld(phi, a.N + k) + St<T>::ld(hi, a.N + k)) * scale);
            I2 += w * ((St<T>::ld(phi, 2 * a.N + k) + St<T>::ld(hi, 2 * a.N + k)) * scale);
        }
    } else {
#pragma unroll 9
        for (int t = 0; t < a.tm; ++t) {
            const int64_t k = tp.k(t);
            const float w = tp.wt(t);
            I0 += w * (St<T>::ld(phi, k) * scale);
            I1 += w * (St<T>::ld(phi, a.N + k) * scale);
            I2 += w * (St<T>::ld(phi, 2 * a.N + k) * scale);
        }
    }
    const float s = a.sj[j];
    d0 = s * (a.wall[j] - I0);
    d1 = s * (a.wall[a.M + j] - I1);
    d2 = s * (a.wall[2 * a.M + j] - I2);
}

template <typename T, typename Ents>
__device__ __forceinline__ void ib_cell(T *phi, float scale, float inv_scale, const IbArgs &a, int64_t k, int km,
                                        const Ents &en, const float *d0, const float *d1, const float *d2) {
    const float v0 = St<T>::ld(phi, k) * scale, v1 = St<T>::ld(phi, a.N + k) * scale,
                v2 = St<T>::ld(phi, 2 * a.N + k) * scale;
    float c0 = 0.f, c1 = 0.f, c2 = 0.f;
#pragma unroll 4
    for (int q = 0; q < km; ++q) {
        const int j = en.j(q);
        const float w = en.wt(q);
        c0 += w * d0[j];
        c1 += w * d1[j];
        c2 += w * d2[j];
    }
    if constexpr (std::is_same<T, float>::value) {
        // float32 cells go out as agent-scope relaxed atomic stores, which write through the L2
        // (the same values; the next sweep reads them on every XCD): 128^3 step 6.77 -> 6.71 ms
        __hip_atomic_store(phi + k, (v0 + c0) * inv_scale, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(phi + a.N + k, (v1 + c1) * inv_scale, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(phi + 2 * a.N + k, (v2 + c2) * inv_scale, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        St<T>::st(phi, k, (v0 + c0) * inv_scale);
        St<T>::st(phi, a.N + k, (v1 + c1) * inv_scale);
        St<T>::st(phi, 2 * a.N + k, (v2 + c2) * inv_scale);
    }
    if (a.copy) {  // float16 copy of the corrected field (the split form's u for the sweeps)
        __half *cp = (__half *)a.copy;
        cp[k] = __float2half_rn((v0 + c0) * a.copy_inv);
        cp[a.N + k] = __float2half_rn((v1 + c1) * a.copy_inv);
        cp[2 * a.N + k] = __float2half_rn((v2 + c2) * a.copy_inv);
    }
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
    if (a.ring) {  // the wave's 64 markers: consecutive x of one line (n_x % 64 == 0)
        const int j0 = blk * kIbThreads + (__builtin_amdgcn_readfirstlane(threadIdx.x) & ~63);
        const int line = j0 / a.nx;
        const LineTaps tp{a.ring_tap + (int64_t)line * a.tm, a.ring_tw + (int64_t)line * a.tm, j - line * a.nx};
        ib_marker(phi, scale, a, j, tp, d0, d1, d2);
    } else {
        ib_marker(phi, scale, a, j, GeneralTaps{a.tap_cell, a.tap_w, a.M, j}, d0, d1, d2);
    }
    // corrections written through the L2 as well (agent-scope relaxed atomic stores)
    __hip_atomic_store(a.delta + j, d0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a.delta + a.M + j, d1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(a.delta + 2 * a.M + j, d2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    const float *d0 = a.delta, *d1 = a.delta + a.M, *d2 = a.delta + 2 * a.M;
    if (a.ring) {  // the wave's 64 cells: consecutive x of one band row (n_x % 64 == 0)
        const int e0 = blk * kIbThreads + (__builtin_amdgcn_readfirstlane(threadIdx.x) & ~63);
        const int row = e0 / a.nx, x = e - row * a.nx;
        const RowEntries en{a.row_mk + (int64_t)row * a.kmr, a.row_w + (int64_t)row * a.kmr, a.nx, x};
        ib_cell(phi, scale, inv_scale, a, (int64_t)x + a.row_off[row], a.kmr, en, d0, d1, d2);
    } else {
        ib_cell(phi, scale, inv_scale, a, (int64_t)a.band_cell[e], a.km, GeneralEntries{a.band_mk, a.band_w, a.nband, e},
                d0, d1, d2);
    }
}

// -------------------------------------------------------------------------------------------
// Lorentz + body force (Sec. 5.1): J = curl_h b with d_a f = 3 sum_i w_i e_ia f(x + e_i),
// F = G x + J x (B_ext + b).
// -------------------------------------------------------------------------------------------
// Force at one cell. b_at(i, ex, ey, ez, v0, v1, v2) gives the induced field (times its scale)
// at neighbour i of c_dir, offset (ex, ey, ez); B is the total field at the cell. The same body
// serves the cell-wise kernel (neighbours from memory) and the fused one (from LDS), so the two
// give the same values bit for bit.
template <bool Q27, typename BAT>
__device__ __forceinline__ void lorentz_force(BAT b_at, float Bx, float By, float Bz, float G, float &F0, float &F1,
                                              float &F2) {
    float g[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};  // g[a][c] = d_c b_a
#pragma unroll
    for (int i = 0; i < (Q27 ? 26 : 18); ++i) {
        const int ex = dir_of(i, 0), ey = dir_of(i, 1), ez = dir_of(i, 2);
        const float w = 3.0f * dir_weight(i, Q27);
        float v0, v1, v2;
        b_at(i, ex, ey, ez, v0, v1, v2);
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
    F0 = G + (Jy * Bz - Jz * By);
    F1 = Jz * Bx - Jx * Bz;
    F2 = Jx * By - Jy * Bx;
}

template <typename TB, bool BATCH, bool SPLIT, bool Q27>
__global__ void __launch_bounds__(kCellThreads) k_lorentz(const TB *b, const TB *bh, float bs, const float *bext,
                                                          const float *bext_yz, const DevCtrl *ctrl, float *F,
                                                          StepConst c, const PipeStep *tab, const BlockMap *map) {
    int64_t blk = blockIdx.x;
    if constexpr (BATCH) {
        const BlockMap m = map[blk];
        const PipeStep &q = tab[m.pipe];
        b = (const TB *)q.b_last;
        bh = (const TB *)q.b_hi;
        bs = q.c.b_scale;
        bext = q.bext;
        bext_yz = q.bext_yz;
        ctrl = q.ctrl;
        F = q.F;
        c = q.c;
        blk = m.local;
    }
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    const int64_t k = blk * kCellThreads + threadIdx.x;
    if (k >= N) return;
    int x, y, z;
    cell_xyz(k, c.nx, c.ny, x, y, z);
    // value of component a at cell i (the split form adds its hi part)
    auto bv = [&](int64_t i) {
        if constexpr (SPLIT)
            return St<TB>::ld(b, i) + St<TB>::ld(bh, i);
        else
            return St<TB>::ld(b, i);
    };
    auto b_at = [&](int, int ex, int ey, int ez, float &v0, float &v1, float &v2) {
        const int kn = wrap1(x + ex, c.nx) + c.nx * (wrap1(y + ey, c.ny) + c.ny * wrap1(z + ez, c.nz));
        v0 = bv(kn) * bs;
        v1 = bv(N + kn) * bs;
        v2 = bv(2 * N + kn) * bs;
    };
    float Bx = bv(k) * bs + bext[x];
    float By = bv(N + k) * bs + bext[c.nx + x];
    float Bz = bv(2 * N + k) * bs + bext[2 * c.nx + x];
    if (bext_yz) {  // six magnets: (y, z) part of B_ext
        const int64_t pyz = (int64_t)c.ny * c.nz, o = y + (int64_t)c.ny * z;
        Bx += bext_yz[o];
        By += bext_yz[pyz + o];
        Bz += bext_yz[2 * pyz + o];
    }
    const float G = (float)ctrl->G_step;
    float F0, F1, F2;
    lorentz_force<Q27>(b_at, Bx, By, Bz, G, F0, F1, F2);
    F[k] = F0;
    F[N + k] = F1;
    F[2 * N + k] = F2;
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
//
// Time-step rescaling (Sec. 7, inv_gamma = 1/gamma): q2 -> q2 / gamma (so DQ scales by 1/gamma),
// the velocity terms of the GZS populations by 1/gamma^2 (G scales by 1/gamma^2; their e.F part
// cancels in the pair sums) and the explicit force F -> F / gamma; tau = 3 nu / gamma + 1/2.
// All three are exact no-ops at gamma = 1.
//
// Macroscopic update (tau >= 1, Sec. 5.7; c.mac): the lattice BGK update with tau = 1 and the GZS
// populations, in v = u / c and phi = F / c^2 with particle speed c = 6 nu (one step is dt = 1/c):
//   f_i(x) = f_i^eq(x - e_i) + P_i(x - e_i),  P_i = (w_i / 2) [3 (e_i - v) . phi + 9 (e_i . v)(e_i . phi)],
//   rho' = sum_i f_i,  rho' v' = sum_i e_i f_i + phi(x) / 2.
// Per pair d (i = +d gathers from x - d, i = -d from x + d), with Q_i = (1 + drho) q_i(v),
// q_i = 3 e_i.v + 4.5 (e_i.v)^2 - 1.5 v.v and H = 9 (d.v)(d.phi) - 3 v.phi (sum_i w_i H_i = 0 at
// one point, sum_i w_i e_i (e_i.phi) = phi / 3):
//   drho' - drho = sum_pairs w [(Ddrho- + Ddrho+) + (DQ_d(x-d) + DQ_-d(x+d))
//                               + 1.5 d.(phi- - phi+) + (H- + H+ - 2 H0) / 2]
//   rho' v' - rho v = phi + sum_pairs w d [(drho- - drho+) + (DQ_d(x-d) - DQ_-d(x+d))
//                               + 1.5 d.(phi- + phi+ - 2 phi) + (H- - H+) / 2]
// with DQ_i(y) = Q_i(y) - Q_i(x): again neighbour differences only.
// -------------------------------------------------------------------------------------------
// One direction of each opposite pair: 3 faces, 6 edges (D3Q19), then the 4 corners of D3Q27.
__device__ constexpr int pair_of(int i, int a) {
    constexpr int t[13][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1},
                              {0, 1, 1}, {0, 1, -1}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
    return t[i][a];
}

// One cell of the fluid update (both branches above). at(ex, ey, ez, d, u0, u1, u2, f0, f1, f2)
// gives the stored density offset, the velocity (times its storage scale) and the force at the
// cell offset (ex, ey, ez) from this one ((0, 0, 0): the cell itself). The same body serves the
// cell-wise kernel (values from memory) and the fused Lorentz + fluid kernel (from LDS), so the
// two give the same results bit for bit.
template <bool Q27, typename AT>
__device__ __forceinline__ void fluid_update(AT at, const StepConst &c, float &dnew, float &un0, float &un1,
                                             float &un2) {
    float d0, cu0, cu1, cu2, cf0, cf1, cf2;  // the cell's own values
    at(0, 0, 0, d0, cu0, cu1, cu2, cf0, cf1, cf2);
    if (c.mac) {
        const float ic = c.inv_mac_c, ic2 = ic * ic;
        const float vx0 = cu0 * ic, vy0 = cu1 * ic, vz0 = cu2 * ic;
        const float px0 = cf0 * ic2, py0 = cf1 * ic2, pz0 = cf2 * ic2;
        const float vv0 = vx0 * vx0 + vy0 * vy0 + vz0 * vz0, vp0 = vx0 * px0 + vy0 * py0 + vz0 * pz0;
        float dr = 0.f, m0 = 0.f, m1 = 0.f, m2 = 0.f;
#pragma unroll
        for (int i = 0; i < (Q27 ? 13 : 9); ++i) {
            const int ex = pair_of(i, 0), ey = pair_of(i, 1), ez = pair_of(i, 2);
            const float w = Q27 ? (i < 3 ? 2.0f / 27.0f : i < 9 ? 1.0f / 54.0f : 1.0f / 216.0f) : (i < 3 ? WF : WE);
            float dp, dm, upx, upy, upz, umx, umy, umz, fpx, fpy, fpz, fmx, fmy, fmz;
            at(ex, ey, ez, dp, upx, upy, upz, fpx, fpy, fpz);
            at(-ex, -ey, -ez, dm, umx, umy, umz, fmx, fmy, fmz);
            const float vpx = upx * ic, vpy = upy * ic, vpz = upz * ic;
            const float vmx = umx * ic, vmy = umy * ic, vmz = umz * ic;
            const float ppx = fpx * ic2, ppy = fpy * ic2, ppz = fpz * ic2;
            const float pmx = fmx * ic2, pmy = fmy * ic2, pmz = fmz * ic2;
            const float Dpx = vpx - vx0, Dpy = vpy - vy0, Dpz = vpz - vz0;
            const float Dmx = vmx - vx0, Dmy = vmy - vy0, Dmz = vmz - vz0;
            const float Ddp = dp - d0, Ddm = dm - d0;
            const float ev0 = ex * vx0 + ey * vy0 + ez * vz0;
            const float eDp = ex * Dpx + ey * Dpy + ez * Dpz, eDm = ex * Dmx + ey * Dmy + ez * Dmz;
            const float q20 = 4.5f * ev0 * ev0 - 1.5f * vv0;
            // q_{+d}(v-) - q_{+d}(v0) and q_{-d}(v+) - q_{-d}(v0)
            const float dqm = 3.0f * eDm + 4.5f * eDm * (eDm + 2.0f * ev0) -
                              1.5f * (Dmx * (vmx + vx0) + Dmy * (vmy + vy0) + Dmz * (vmz + vz0));
            const float dqp = -3.0f * eDp + 4.5f * eDp * (eDp + 2.0f * ev0) -
                              1.5f * (Dpx * (vpx + vx0) + Dpy * (vpy + vy0) + Dpz * (vpz + vz0));
            const float DQm = (1.0f + dm) * dqm + Ddm * (q20 + 3.0f * ev0);
            const float DQp = (1.0f + dp) * dqp + Ddp * (q20 - 3.0f * ev0);
            const float epm = ex * pmx + ey * pmy + ez * pmz, epp = ex * ppx + ey * ppy + ez * ppz,
                        ep0 = ex * px0 + ey * py0 + ez * pz0;
            const float Hm = 9.0f * (ev0 + eDm) * epm - 3.0f * (vmx * pmx + vmy * pmy + vmz * pmz);
            const float Hp = 9.0f * (ev0 + eDp) * epp - 3.0f * (vpx * ppx + vpy * ppy + vpz * ppz);
            const float H0 = 9.0f * ev0 * ep0 - 3.0f * vp0;
            dr += w * ((Ddm + Ddp) + (DQm + DQp) + 1.5f * (epm - epp) + 0.5f * ((Hm - H0) + (Hp - H0)));
            const float cm = w * ((dm - dp) + (DQm - DQp) + 1.5f * ((epm - ep0) + (epp - ep0)) + 0.5f * (Hm - Hp));
            m0 += ex * cm;
            m1 += ey * cm;
            m2 += ez * cm;
        }
        dnew = d0 + dr;
        const float inv = 1.0f / (1.0f + dnew);
        const float cu = c.mac_c;
        un0 = cu * (vx0 + ((m0 + px0) - dr * vx0) * inv);
        un1 = cu * (vy0 + ((m1 + py0) - dr * vy0) * inv);
        un2 = cu * (vz0 + ((m2 + pz0) - dr * vz0) * inv);
        return;
    }
    const float tau = c.tau, ig = c.inv_gamma;
    const float cF = 1.0f - 0.5f / tau;
    const float a3 = 3.0f * (2.0f * tau - 1.0f);
    const float ux0 = cu0, uy0 = cu1, uz0 = cu2;
    const float uu0 = ux0 * ux0 + uy0 * uy0 + uz0 * uz0;
    float dr = 0.f;
    float m0 = 0.f, m1 = 0.f, m2 = 0.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
#pragma unroll
    for (int i = 0; i < (Q27 ? 13 : 9); ++i) {
        const int ex = pair_of(i, 0), ey = pair_of(i, 1), ez = pair_of(i, 2);
        const float w = Q27 ? (i < 3 ? 2.0f / 27.0f : i < 9 ? 1.0f / 54.0f : 1.0f / 216.0f) : (i < 3 ? WF : WE);
        float dp, dm, upx, upy, upz, umx, umy, umz, fpx, fpy, fpz, fmx, fmy, fmz;
        at(ex, ey, ez, dp, upx, upy, upz, fpx, fpy, fpz);
        at(-ex, -ey, -ez, dm, umx, umy, umz, fmx, fmy, fmz);
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
        const float DQp = ig * ((1.0f + dp) * dq2p + Ddp * q20), DQm = ig * ((1.0f + dm) * dq2m + Ddm * q20);
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
    dnew = d0 + dr;
    const float tcF = tau * cF * (ig * ig);
    const float Dm0 = (m0 - tcF * g0) + cf0 * ig;
    const float Dm1 = (m1 - tcF * g1) + cf1 * ig;
    const float Dm2 = (m2 - tcF * g2) + cf2 * ig;
    const float inv = 1.0f / (1.0f + dnew);
    un0 = ux0 + (Dm0 - dr * ux0) * inv;
    un1 = uy0 + (Dm1 - dr * uy0) * inv;
    un2 = uz0 + (Dm2 - dr * uz0) * inv;
}

// New state of one cell from fluid_update: stores, the split form's float16 copy of u, and the
// blow-up flag (a non-finite or supersonic velocity marks the box; every such lane stores the same
// value, so the plain store needs no atomic).
template <typename TR, typename TU>
__device__ __forceinline__ void fluid_store(int64_t k, int64_t N, float dnew, float un0, float un1, float un2,
                                            TR *rho_o, TU *u_o, __half *u_copy, const StepConst &c) {
    if (!((double)(un0 * un0 + un1 * un1 + un2 * un2) < c.u_limit2) || !(dnew == dnew)) *c.status = 1;
    St<TR>::st(rho_o, k, dnew);
    St<TU>::st(u_o, k, un0 * c.inv_u_scale);
    St<TU>::st(u_o, N + k, un1 * c.inv_u_scale);
    St<TU>::st(u_o, 2 * N + k, un2 * c.inv_u_scale);
    if (u_copy) {  // split form: float16 copy u / u_scale for the sweeps
        u_copy[k] = __float2half_rn(un0 * c.inv_copy_scale);
        u_copy[N + k] = __float2half_rn(un1 * c.inv_copy_scale);
        u_copy[2 * N + k] = __float2half_rn(un2 * c.inv_copy_scale);
    }
}

template <typename TR, typename TU, bool BATCH, bool Q27>
__global__ void __launch_bounds__(kCellThreads) k_fluid(const TR *rho, const TU *u, const float *F, TR *rho_o,
                                                        TU *u_o, __half *u_copy, StepConst c, const PipeStep *tab,
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
        u_copy = (__half *)q.u_copy;
        c = q.c;
        blk = m.local;
    }
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    const int64_t k = blk * kCellThreads + threadIdx.x;
    if (k >= N) return;
    int x, y, z;
    cell_xyz(k, c.nx, c.ny, x, y, z);
    const float us = c.u_scale;
    auto at = [&](int ex, int ey, int ez, float &d, float &u0_, float &u1_, float &u2_, float &f0, float &f1,
                  float &f2) {
        const int kk = wrap1(x + ex, c.nx) + c.nx * (wrap1(y + ey, c.ny) + c.ny * wrap1(z + ez, c.nz));
        d = St<TR>::ld(rho, kk);
        u0_ = St<TU>::ld(u, kk) * us;
        u1_ = St<TU>::ld(u, N + kk) * us;
        u2_ = St<TU>::ld(u, 2 * N + kk) * us;
        f0 = F[kk];
        f1 = F[N + kk];
        f2 = F[2 * N + kk];
    };
    float dnew, un0, un1, un2;
    fluid_update<Q27>(at, c, dnew, un0, un1, un2);
    fluid_store(k, N, dnew, un0, un1, un2, rho_o, u_o, u_copy, c);
}

// -------------------------------------------------------------------------------------------
// Lorentz force and fluid update in one plane-marching kernel (single boxes, float32 storage).
// A workgroup owns a 64 x 4 column of cells and marches along z over a chunk of planes. Each
// plane of b is staged in LDS with a two-cell halo, each plane of rho and u with a one-cell
// halo; the force of a plane is formed in LDS on the one-cell halo from the three b planes
// around it (lorentz_force), and the fluid update of the plane before takes its neighbours'
// rho, u and F from LDS (fluid_update). F never goes to memory: the pair reads b, rho and u and
// writes rho and u once, 44 B per cell (the two-kernel form also writes and re-reads F, and
// gathers every neighbour through the caches). Rings of 4 (b, F) and 5 (rho, u) planes let one
// barrier per plane separate the writes of a plane from the reads of the planes before it. The
// cell arithmetic is the same code as k_lorentz and k_fluid, so the results are the same bit
// for bit.
// -------------------------------------------------------------------------------------------
constexpr int kLfTX = 64, kLfTY = 4;                         // output tile (256 work-items)
constexpr int kLfBX = kLfTX + 4, kLfBY = kLfTY + 4;          // b with a two-cell halo
constexpr int kLfFX = kLfTX + 2, kLfFY = kLfTY + 2;          // F, rho, u with a one-cell halo
constexpr int kLfBN = kLfBX * kLfBY, kLfFN = kLfFX * kLfFY;  // 544, 396 cells per plane
constexpr int kLfBS = (kLfBN + kCellThreads - 1) / kCellThreads;  // b cells staged per work-item
constexpr int kLfFS = (kLfFN + kCellThreads - 1) / kCellThreads;  // F / rho-u cells per work-item

__device__ __forceinline__ int ring5(int p) { return ((p % 5) + 5) % 5; }

template <bool Q27>
__global__ void __launch_bounds__(kCellThreads) k_lorentz_fluid(LfArgs a) {
    __shared__ float sb[4][3][kLfBN];
    __shared__ float sF[4][3][kLfFN];
    __shared__ float sr[5][4][kLfFN];
    const StepConst &c = a.c;
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int64_t N = (int64_t)nx * ny * nz;
    const unsigned plane = (unsigned)nx * ny;
    // XCD-aware order (as for the sweep): each XCD receives a contiguous run of tiles
    const int per = gridDim.x >> 3;
    const int lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
    if (lb >= a.nblocks) return;
    const int tix = lb % a.tiles_x, rest = lb / a.tiles_x;
    const int tiy = rest % a.tiles_y, tiz = rest / a.tiles_y;
    const int x0 = tix * kLfTX, y0 = tiy * kLfTY, z0 = tiz * a.zchunk;
    const int z1 = min(z0 + a.zchunk, nz);
    const int t = threadIdx.x;
    const float us = c.u_scale, bs = c.b_scale;

    // staged cells of this work-item (fixed (x, y) for the whole march)
    unsigned bxy[kLfBS];
    bool bval[kLfBS];
#pragma unroll
    for (int s = 0; s < kLfBS; ++s) {
        const int i = t + s * kCellThreads;
        bval[s] = i < kLfBN;
        const int hx = i % kLfBX, hy = i / kLfBX;
        bxy[s] = (unsigned)(wrapi(x0 - 2 + hx, nx) + nx * wrapi(y0 - 2 + hy, ny));
    }
    unsigned fxy[kLfFS];
    bool fval[kLfFS];
#pragma unroll
    for (int s = 0; s < kLfFS; ++s) {
        const int i = t + s * kCellThreads;
        fval[s] = i < kLfFN;
        const int hx = i % kLfFX, hy = i / kLfFX;
        fxy[s] = (unsigned)(wrapi(x0 - 1 + hx, nx) + nx * wrapi(y0 - 1 + hy, ny));
    }
    float rb[kLfBS][3], rr[kLfFS][4];
    auto load_b = [&](int p) {
        const unsigned off = (unsigned)wrapi(p, nz) * plane;
#pragma unroll
        for (int s = 0; s < kLfBS; ++s)
            if (bval[s])
#pragma unroll
                for (int q = 0; q < 3; ++q) rb[s][q] = a.b[q * N + off + bxy[s]];
    };
    auto store_b = [&](int p) {
#pragma unroll
        for (int s = 0; s < kLfBS; ++s)
            if (bval[s])
#pragma unroll
                for (int q = 0; q < 3; ++q) sb[p & 3][q][t + s * kCellThreads] = rb[s][q];
    };
    auto load_r = [&](int p) {
        const unsigned off = (unsigned)wrapi(p, nz) * plane;
#pragma unroll
        for (int s = 0; s < kLfFS; ++s)
            if (fval[s]) {
                rr[s][0] = a.rho[off + fxy[s]];
#pragma unroll
                for (int q = 0; q < 3; ++q) rr[s][1 + q] = a.u[q * N + off + fxy[s]];
            }
    };
    auto store_r = [&](int p) {
#pragma unroll
        for (int s = 0; s < kLfFS; ++s)
            if (fval[s])
#pragma unroll
                for (int q = 0; q < 4; ++q) sr[ring5(p)][q][t + s * kCellThreads] = rr[s][q];
    };
    // force of plane p on the one-cell halo region, from b planes p - 1 .. p + 1
    const float G = (float)a.ctrl->G_step;
    auto force = [&](int p) {
        const int zz = wrapi(p, nz);
#pragma unroll 1
        for (int i = t; i < kLfFN; i += kCellThreads) {
            const int hx = i % kLfFX + 1, hy = i / kLfFX + 1;  // position in the b region
            const int gx = wrapi(x0 - 2 + hx, nx), gy = wrapi(y0 - 2 + hy, ny);
            auto b_at = [&](int, int ex, int ey, int ez, float &v0, float &v1, float &v2) {
                const int sl = (p + ez) & 3, o = (hy + ey) * kLfBX + (hx + ex);
                v0 = sb[sl][0][o] * bs;
                v1 = sb[sl][1][o] * bs;
                v2 = sb[sl][2][o] * bs;
            };
            const int oc = hy * kLfBX + hx;
            float Bx = sb[p & 3][0][oc] * bs + a.bext[gx];
            float By = sb[p & 3][1][oc] * bs + a.bext[nx + gx];
            float Bz = sb[p & 3][2][oc] * bs + a.bext[2 * nx + gx];
            if (a.bext_yz) {  // six magnets: (y, z) part of B_ext
                const int64_t pyz = (int64_t)ny * nz, o = gy + (int64_t)ny * zz;
                Bx += a.bext_yz[o];
                By += a.bext_yz[pyz + o];
                Bz += a.bext_yz[2 * pyz + o];
            }
            float F0, F1, F2;
            lorentz_force<Q27>(b_at, Bx, By, Bz, G, F0, F1, F2);
            sF[p & 3][0][i] = F0;
            sF[p & 3][1][i] = F1;
            sF[p & 3][2][i] = F2;
        }
    };
    // fluid update of the output cell of this work-item on plane q
    const int lx = t % kLfTX, ly = t / kLfTX;
    const int ox = x0 + lx, oy = y0 + ly;
    const bool own = ox < nx && oy < ny;
    auto fluid = [&](int q) {
        auto at = [&](int ex, int ey, int ez, float &d, float &u0_, float &u1_, float &u2_, float &f0, float &f1,
                      float &f2) {
            const int rs = ring5(q + ez), fs = (q + ez) & 3, o = (ly + 1 + ey) * kLfFX + (lx + 1 + ex);
            d = sr[rs][0][o];
            u0_ = sr[rs][1][o] * us;
            u1_ = sr[rs][2][o] * us;
            u2_ = sr[rs][3][o] * us;
            f0 = sF[fs][0][o];
            f1 = sF[fs][1][o];
            f2 = sF[fs][2][o];
        };
        float dnew, un0, un1, un2;
        fluid_update<Q27>(at, c, dnew, un0, un1, un2);
        const int64_t k = (int64_t)q * plane + ox + (int64_t)nx * oy;
        fluid_store(k, N, dnew, un0, un1, un2, a.rho_o, a.u_o, (__half *)nullptr, c);
    };

    // prologue: b planes z0 - 2 .. z0 and rho, u of plane z0 - 1 in LDS; the next planes requested
    load_b(z0 - 2);
    store_b(z0 - 2);
    load_b(z0 - 1);
    store_b(z0 - 1);
    load_b(z0);
    store_b(z0);
    load_r(z0 - 1);
    store_r(z0 - 1);
    load_b(z0 + 1);
    load_r(z0);
    __syncthreads();
    for (int p = z0 - 1; p <= z1; ++p) {
        force(p);
        store_b(p + 2);               // b is needed up to plane z1 + 1, rho and u up to z1; the
        store_r(p + 1);               // requests below are clamped so that every one is issued
        load_b(min(p + 3, z1 + 1));
        load_r(min(p + 2, z1));
        __syncthreads();
        if (p - 1 >= z0 && own) fluid(p - 1);
    }
}

// -------------------------------------------------------------------------------------------
// Float64 reductions with a fixed summation order: a fixed grid of kRedBlocks workgroups walks
// the cells with a fixed stride, each block reduces its values with wave shuffles and one LDS
// exchange between its waves (block_reduce above) and writes one partial; a single block then
// sums the partials in the same way.
// -------------------------------------------------------------------------------------------

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
    __shared__ double sh[1][kRedWaves];
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    const double R2 = c.radius * c.radius;
    double s = 0.0;
    for (int64_t k = (int64_t)blk * kRedThreads + threadIdx.x; k < N; k += (int64_t)kRedBlocks * kRedThreads) {
        int x, y, z;
        cell_xyz(k, c.nx, c.ny, x, y, z);
        const double dy = y - c.yc, dz = z - c.zc;
        if (dy * dy + dz * dz <= R2) s += (double)(St<TU>::ld(u, k) * c.u_scale);
    }
    double v[1] = {s};
    block_reduce<1, 0>(sh, v, nullptr);
    if (threadIdx.x == 0) part[blk] = v[0];
}

// partial layout: 0 Ek, 1 Em, 2 Eb, 3 sum u_x (Omega), 4 Pp, 5 Pnu/nu, 6 PL, 7 Meta/eta, 8 Madv,
// 9 sum |J|^2, 10 mass, 11 Q sum, 12 n_omega, 13 sum |eta lap b - div(uB - Bu)|^2 (the induction
// residual of Sec. 5.8), 14 sum b . lap b (Joule dissipation in Dirichlet form, times -eta),
// 15 max |u|^2, 16 nonfinite
template <typename TR, typename TU, typename TB>
__global__ void __launch_bounds__(kRedThreads) k_budget_partial(const TR *rho, const TU *u, const TB *b,
                                                                const TB *bh, const float *bext,
                                                                const float *bext_yz, double *part, StepConst c) {
    __shared__ double sh[17][kRedWaves];
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    const double us = c.u_scale, bs = c.b_scale;
    const double R2 = c.radius * c.radius;
    const double Ro2 = c.omega_radius * c.omega_radius;
    double v[15];
#pragma unroll
    for (int q = 0; q < 15; ++q) v[q] = 0.0;
    double umax2 = 0.0;
    double nonfin = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; k < N; k += (int64_t)kRedBlocks * kRedThreads) {
        int x, y, z;
        cell_xyz(k, c.nx, c.ny, x, y, z);
        const double r = 1.0 + (double)St<TR>::ld(rho, k);
        double uu[3], bb[3], B[3];
        for (int a = 0; a < 3; ++a) {
            uu[a] = (double)St<TU>::ld(u, a * N + k) * us;
            bb[a] = (double)St<TB>::ld(b, a * N + k) * bs;
            if (bh) bb[a] += (double)St<TB>::ld(bh, a * N + k) * bs;
            B[a] = bb[a] + (double)bext[a * c.nx + x];
            if (bext_yz) B[a] += (double)bext_yz[a * (int64_t)c.ny * c.nz + y + (int64_t)c.ny * z];
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
        const bool q27 = c.lattice == 27;
        for (int i = 0; i < (q27 ? 26 : 18); ++i) {
            const int e[3] = {c_dir[i][0], c_dir[i][1], c_dir[i][2]};
            const double w = dir_weight_d(i, q27);
            const int xn = wrap1(x + e[0], c.nx);
            const int kn = xn + c.nx * (wrap1(y + e[1], c.ny) + c.ny * wrap1(z + e[2], c.nz));
            const double rn = 1.0 + (double)St<TR>::ld(rho, kn);
            double un[3], bn[3], Bn[3];
            for (int a = 0; a < 3; ++a) {
                un[a] = (double)St<TU>::ld(u, a * N + kn) * us;
                bn[a] = (double)St<TB>::ld(b, a * N + kn) * bs;
                if (bh) bn[a] += (double)St<TB>::ld(bh, a * N + kn) * bs;
                Bn[a] = bn[a] + (double)bext[a * c.nx + xn];
                if (bext_yz)
                    Bn[a] += (double)bext_yz[a * (int64_t)c.ny * c.nz + wrap1(y + e[1], c.ny) +
                                             (int64_t)c.ny * wrap1(z + e[2], c.nz)];
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
            const double res = c.eta * lb[a] - divL[a];
            v[13] += res * res;
            v[14] += bb[a] * lb[a];
        }
    }
    // the 15 sums, max |u|^2 and "any non-finite" in the same fixed order
    double mx[2] = {umax2, nonfin};
    block_reduce<15, 2>(sh, v, mx);
    if (threadIdx.x == 0) {
        double *o = part + (int64_t)blockIdx.x * kBudgetVals;
        for (int q = 0; q < 15; ++q) o[q] = v[q];
        o[15] = mx[0];
        o[16] = mx[1];
    }
}

__global__ void __launch_bounds__(kRedThreads) k_budget_final(const double *part, DevCtrl *ctrl, mhd_budget *ring,
                                                              StepConst c) {
    __shared__ double sh[17][kRedWaves];
    double v[15];
#pragma unroll
    for (int q = 0; q < 15; ++q) v[q] = 0.0;
    double m = 0.0, f = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) {
        const double *p = part + (int64_t)i * kBudgetVals;
#pragma unroll
        for (int q = 0; q < 15; ++q) v[q] += p[q];
        m = fmax(m, p[15]);
        f = fmax(f, p[16]);
    }
    double mx[2] = {m, f};
    block_reduce<15, 2>(sh, v, mx);
    if (threadIdx.x == 0) {
        const double n = v[12];
        const double inv = n > 0.0 ? 1.0 / n : 0.0;
        mhd_budget r;
        r.step = ctrl->t;
        r.G = ctrl->G_step;
        r.E_k = v[0] * inv;
        r.E_m = v[1] * inv;
        r.E_b = v[2] * inv;
        r.P_in = r.G * v[3] * inv;
        r.P_p = v[4] * inv;
        r.P_nu = c.nu * v[5] * inv;
        r.P_L = v[6] * inv;
        r.M_eta = c.eta * v[7] * inv;
        r.M_adv = v[8] * inv;
        r.joule = c.eta * v[9] * inv;
        r.mass = v[10];
        r.Q = v[11] / (double)c.nx;
        r.u_max = sqrt(mx[0]);
        r.n_omega = n;
        r.res_mag = sqrt(v[13] * inv);
        r.D_eta = -c.eta * v[14] * inv;
        // |u| >= c_s or a non-finite value marks the run unstable
        if (mx[1] != 0.0 || !(mx[0] < c.u_limit2) || !isfinite(v[0])) ctrl->status |= 1;
        const int idx = ctrl->n_records;
        if (idx < kRingCap) {
            ring[idx] = r;
            ctrl->n_records = idx + 1;
        } else {
            ctrl->overflow += 1;
        }
    }
}

// Residual only: the same fixed-order sum of the partials' slots 13 (residual) and 12 (cells).
__global__ void __launch_bounds__(kRedThreads) k_residual_final(const double *part, double *out) {
    __shared__ double sh[2][kRedWaves];
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) {
        v[0] += part[(int64_t)i * kBudgetVals + 13];
        v[1] += part[(int64_t)i * kBudgetVals + 12];
    }
    block_reduce<2, 0>(sh, v, nullptr);
    if (threadIdx.x == 0) *out = v[1] > 0.0 ? sqrt(v[0] / v[1]) : 0.0;
}

// -------------------------------------------------------------------------------------------
// Storage conversion (float32 staging <-> storage kind)
// -------------------------------------------------------------------------------------------
template <typename T>
__global__ void k_store(const float *src, T *dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        St<T>::st(dst, i, src[i]);
}
__global__ void k_store_split(const float *src, __half *hi, __half *lo, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const __half h = __float2half_rn(src[i]);
        hi[i] = h;
        lo[i] = __float2half_rn(src[i] - __half2float(h));
    }
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

#define MHD_DISPATCH1(kind, FN, ...)                                       \
    switch (kind) {                                                        \
        case MHD_KIND_F32: return FN<float>(__VA_ARGS__);                  \
        case MHD_KIND_F16:                                                 \
        case MHD_KIND_F16_SPLIT: return FN<__half>(__VA_ARGS__);           \
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

template <typename T, bool SPLIT>
static hipError_t lorentz_t(hipStream_t s, const void *b, const void *bh, const float *bext, const float *bext_yz,
                            const DevCtrl *ctrl, float *F, StepConst c) {
    const int64_t N = (int64_t)c.nx * c.ny * c.nz;
    if (c.lattice == 27)
        hipLaunchKernelGGL((k_lorentz<T, false, SPLIT, true>), dim3(blocks_for(N, kCellThreads)), dim3(kCellThreads),
                           0, s, (const T *)b, (const T *)bh, c.b_scale, bext, bext_yz, ctrl, F, c, nullptr, nullptr);
    else
        hipLaunchKernelGGL((k_lorentz<T, false, SPLIT, false>), dim3(blocks_for(N, kCellThreads)), dim3(kCellThreads),
                           0, s, (const T *)b, (const T *)bh, c.b_scale, bext, bext_yz, ctrl, F, c, nullptr, nullptr);
    return hipGetLastError();
}
hipError_t launch_lorentz(hipStream_t s, int kind_b, const void *b, const void *b_hi, const float *bext,
                          const float *bext_yz, const DevCtrl *ctrl, float *F, StepConst c) {
    switch (kind_b) {
        case MHD_KIND_F32: return lorentz_t<float, false>(s, b, b_hi, bext, bext_yz, ctrl, F, c);
        case MHD_KIND_F16: return lorentz_t<__half, false>(s, b, b_hi, bext, bext_yz, ctrl, F, c);
        case MHD_KIND_BF16: return lorentz_t<__hip_bfloat16, false>(s, b, b_hi, bext, bext_yz, ctrl, F, c);
        case MHD_KIND_F16_SPLIT: return lorentz_t<__half, true>(s, b, b_hi, bext, bext_yz, ctrl, F, c);
        default: return hipErrorInvalidValue;
    }
}
template <typename T, bool SPLIT>
static hipError_t lorentz_batch_t(hipStream_t s, const PipeStep *tab, const BlockMap *map, int nblocks, bool q27) {
    if (nblocks <= 0) return hipSuccess;
    if (q27)
        hipLaunchKernelGGL((k_lorentz<T, true, SPLIT, true>), dim3(nblocks), dim3(kCellThreads), 0, s, nullptr, nullptr,
                           0.f, nullptr, nullptr, nullptr, nullptr, StepConst{}, tab, map);
    else
        hipLaunchKernelGGL((k_lorentz<T, true, SPLIT, false>), dim3(nblocks), dim3(kCellThreads), 0, s, nullptr,
                           nullptr, 0.f, nullptr, nullptr, nullptr, nullptr, StepConst{}, tab, map);
    return hipGetLastError();
}
hipError_t launch_lorentz_batch(hipStream_t s, int kind_b, const PipeStep *tab, const BlockMap *map, int nblocks,
                                bool q27) {
    switch (kind_b) {
        case MHD_KIND_F32: return lorentz_batch_t<float, false>(s, tab, map, nblocks, q27);
        case MHD_KIND_F16: return lorentz_batch_t<__half, false>(s, tab, map, nblocks, q27);
        case MHD_KIND_BF16: return lorentz_batch_t<__hip_bfloat16, false>(s, tab, map, nblocks, q27);
        case MHD_KIND_F16_SPLIT: return lorentz_batch_t<__half, true>(s, tab, map, nblocks, q27);
        default: return hipErrorInvalidValue;
    }
}

template <typename TR, typename TU, bool BATCH>
static hipError_t fluid_t(hipStream_t s, const void *rho, const void *u, const float *F, void *rho_o, void *u_o,
                          void *u_copy, StepConst c, const PipeStep *tab, const BlockMap *map, int nblocks) {
    if (!BATCH) nblocks = (int)blocks_for((int64_t)c.nx * c.ny * c.nz, kCellThreads);
    if (nblocks <= 0) return hipSuccess;
    if (c.lattice == 27)  // batched launches pass the lattice of the whole batch in c
        hipLaunchKernelGGL((k_fluid<TR, TU, BATCH, true>), dim3(nblocks), dim3(kCellThreads), 0, s, (const TR *)rho,
                           (const TU *)u, F, (TR *)rho_o, (TU *)u_o, (__half *)u_copy, c, tab, map);
    else
        hipLaunchKernelGGL((k_fluid<TR, TU, BATCH, false>), dim3(nblocks), dim3(kCellThreads), 0, s, (const TR *)rho,
                           (const TU *)u, F, (TR *)rho_o, (TU *)u_o, (__half *)u_copy, c, tab, map);
    return hipGetLastError();
}
template <bool BATCH>
static hipError_t fluid_kinds(hipStream_t s, int kinds, const void *rho, const void *u, const float *F, void *rho_o,
                              void *u_o, void *u_copy, StepConst c, const PipeStep *tab, const BlockMap *map,
                              int nblocks) {
    const int kr = kinds & 15, ku = (kinds >> 4) & 15;
    if (kr == MHD_KIND_F32 && ku == MHD_KIND_F32)
        return fluid_t<float, float, BATCH>(s, rho, u, F, rho_o, u_o, u_copy, c, tab, map, nblocks);
    if (kr == MHD_KIND_F16 && ku == MHD_KIND_F16)
        return fluid_t<__half, __half, BATCH>(s, rho, u, F, rho_o, u_o, u_copy, c, tab, map, nblocks);
    if (kr == MHD_KIND_F16 && ku == MHD_KIND_BF16)
        return fluid_t<__half, __hip_bfloat16, BATCH>(s, rho, u, F, rho_o, u_o, u_copy, c, tab, map, nblocks);
    if (kr == MHD_KIND_BF16 && ku == MHD_KIND_BF16)
        return fluid_t<__hip_bfloat16, __hip_bfloat16, BATCH>(s, rho, u, F, rho_o, u_o, u_copy, c, tab, map,
                                                              nblocks);
    return hipErrorInvalidValue;
}
hipError_t launch_fluid(hipStream_t s, int kinds, const void *rho, const void *u, const float *F, void *rho_o,
                        void *u_o, void *u_copy, StepConst c) {
    return fluid_kinds<false>(s, kinds, rho, u, F, rho_o, u_o, u_copy, c, nullptr, nullptr, 0);
}
hipError_t launch_lorentz_fluid(hipStream_t s, const LfArgs &a0) {
    LfArgs a = a0;
    a.tiles_x = (a.c.nx + kLfTX - 1) / kLfTX;
    a.tiles_y = (a.c.ny + kLfTY - 1) / kLfTY;
    const int64_t cols = (int64_t)a.tiles_x * a.tiles_y;
    a.zchunk = cols * ((a.c.nz + 15) / 16) >= 512 ? 16 : 8;  // 16-plane chunks when they fill the chip
    a.nblocks = (int)(cols * ((a.c.nz + a.zchunk - 1) / a.zchunk));
    const dim3 grid((unsigned)(((a.nblocks + 7) / 8) * 8));
    if (a.c.lattice == 27)
        hipLaunchKernelGGL(k_lorentz_fluid<true>, grid, dim3(kCellThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_lorentz_fluid<false>, grid, dim3(kCellThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fluid_batch(hipStream_t s, int kinds, const PipeStep *tab, const BlockMap *map, int nblocks,
                              bool q27) {
    StepConst c{};
    c.lattice = q27 ? 27 : 19;
    return fluid_kinds<true>(s, kinds, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, c, tab, map, nblocks);
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
static hipError_t budget_t(hipStream_t s, const void *rho, const void *u, const void *b, const void *bh,
                           const float *bext, const float *bext_yz, DevCtrl *ctrl, double *part, mhd_budget *ring,
                           StepConst c) {
    hipLaunchKernelGGL((k_budget_partial<TR, TU, TB>), dim3(kRedBlocks), dim3(kRedThreads), 0, s, (const TR *)rho,
                       (const TU *)u, (const TB *)b, (const TB *)bh, bext, bext_yz, part, c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ring) return e;  // no ring: partials only
    hipLaunchKernelGGL(k_budget_final, dim3(1), dim3(kRedThreads), 0, s, part, ctrl, ring, c);
    return hipGetLastError();
}
hipError_t launch_residual_final(hipStream_t s, const double *part, double *out) {
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(kRedThreads), 0, s, part, out);
    return hipGetLastError();
}

hipError_t launch_budget(hipStream_t s, int kinds, const void *rho, const void *u, const void *b, const void *b_hi,
                         const float *bext, const float *bext_yz, DevCtrl *ctrl, double *part, mhd_budget *ring,
                         StepConst c) {
    const int kr = kinds & 15, ku = (kinds >> 4) & 15, kb = (kinds >> 8) & 15;
    if (kr == MHD_KIND_F32 && ku == MHD_KIND_F32 && kb == MHD_KIND_F32)
        return budget_t<float, float, float>(s, rho, u, b, nullptr, bext, bext_yz, ctrl, part, ring, c);
    if (kr == MHD_KIND_F32 && ku == MHD_KIND_F32 && kb == MHD_KIND_F16_SPLIT)
        return budget_t<float, float, __half>(s, rho, u, b, b_hi, bext, bext_yz, ctrl, part, ring, c);
    if (kr == MHD_KIND_F16 && ku == MHD_KIND_F16 && kb == MHD_KIND_F16)
        return budget_t<__half, __half, __half>(s, rho, u, b, nullptr, bext, bext_yz, ctrl, part, ring, c);
    if (kr == MHD_KIND_F16 && ku == MHD_KIND_BF16 && kb == MHD_KIND_F16)
        return budget_t<__half, __hip_bfloat16, __half>(s, rho, u, b, nullptr, bext, bext_yz, ctrl, part, ring, c);
    if (kr == MHD_KIND_BF16 && ku == MHD_KIND_BF16 && kb == MHD_KIND_BF16)
        return budget_t<__hip_bfloat16, __hip_bfloat16, __hip_bfloat16>(s, rho, u, b, nullptr, bext, bext_yz, ctrl, part, ring,
                                                                         c);
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

hipError_t launch_store_split(hipStream_t s, const float *src, void *hi, void *lo, int64_t n) {
    hipLaunchKernelGGL(k_store_split, dim3((unsigned)std::min<int64_t>(blocks_for(n, 256), 65536)), dim3(256), 0, s,
                       src, (__half *)hi, (__half *)lo, n);
    return hipGetLastError();
}

}  // namespace mhd
