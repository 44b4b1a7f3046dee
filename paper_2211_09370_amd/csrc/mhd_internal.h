// Internal declarations shared by the host runtime and the gfx950 kernels of mhdlbm.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mhdlbm.h"

namespace mhd {

// Device-side control block: step counter, body force, status and budget-ring bookkeeping.
struct DevCtrl {
    double G;          // controlled body force (state of the integral law)
    double G_step;     // body force used by the step in flight
    int64_t t;         // steps completed
    int32_t status;    // bit 0: unstable
    int32_t n_records; // budget records written since the host last drained the ring
    int32_t overflow;  // records dropped because the ring was full
    int32_t pad[9];
};

// Scalar parameters the step kernels read (copied by value into every launch).
struct StepConst {
    int nx, ny, nz;
    float kappa;       // 1 / (2 eta)
    float tau;         // 3 nu / gamma + 1/2
    float inv_gamma;   // 1 / gamma of the rescaled fluid update (1: none)
    int mac;           // 1: macroscopic tau = 1 fluid update with particle speed mac_c = 6 nu
    float mac_c, inv_mac_c;
    double u_limit2;   // |u|^2 at or above which the state is flagged unstable (c_s^2)
    int32_t *status;   // the box's DevCtrl::status: the fluid update stores 1 there when a new
                       // velocity is non-finite or reaches c_s
    float u_scale, inv_u_scale, b_scale, inv_b_scale;
    float copy_scale, inv_copy_scale;  // split form: scale of the float16 copy of u
    float omega;                       // 1 / alpha of the accelerated magnetic iteration
    int lattice;                       // 19 or 27
    double nu, eta;
    double G0, G1, period;
    double yc, zc, radius;
    double omega_radius;  // budget region r < omega_radius
    int flow_control;
    double u_target, k_c;
};

constexpr int kRedBlocks = 1024;   // fixed grid of the float64 reductions (fixed summation order)
constexpr int kRedThreads = 256;
constexpr int kBudgetVals = 17;    // per-block partial sums of a budget pass
constexpr int kRingCap = 4096;     // budget records held on the device
constexpr int kResCap = 4096;      // residual values of one mhd_mag_residual_curve call

// Launch wrappers implemented in mhd_kernels.hip. Every pointer is a device pointer.
struct SweepLaunch {
    int tx, ty, zchunk;  // tile shape and z extent of one workgroup
    int pair;            // 1: two x cells per lane (n_x a multiple of 128); ty = rows per tile
    int byz = 0;         // 1: add the (y, z) table of B_ext (six magnets) while staging
    int q27 = 0;         // 1: D3Q27 weights
};

// Arguments of one magnetic sweep launch over one box.
struct SweepArgs {
    const void *u;      // velocity as the sweep reads it (the float16 copy in the split form)
    const void *b;      // b (split form: its lo part)
    void *bo;           // output b (split form: lo part)
    const void *bh;     // split form: hi part of b (else NULL)
    void *bho;          // split form, first sweep of a step: re-split hi output (else NULL)
    const float *bext;  // 3 x nx
    const float *bext_yz;  // 3 x (ny nz) table added to bext (six magnets), else NULL
    int nx, ny, nz;
    int tiles_x, tiles_y, nzc, zchunk, nblocks;
    float kappa, u_scale, b_scale, inv_b_scale;
    float omega;        // b' = b + omega (S(b) - b); 1 for the plain sweep
    int q27;            // 1: D3Q27 lattice
};
// Sweep arguments of a box for tile choice L (tile counts and workgroup count filled in).
SweepArgs make_sweep_args(const void *u, const void *b, void *bo, const float *bext, StepConst c, SweepLaunch L);

hipError_t launch_ctrl_begin(hipStream_t s, DevCtrl *ctrl, StepConst c);
hipError_t launch_step_end(hipStream_t s, DevCtrl *ctrl, const double *flow_part, StepConst c,
                           double inv_count);
// One sweep with arguments a (from make_sweep_args, split-form fields filled in by the caller).
// e0 / e1 (optional): events stamped at the start and end of the sweep kernel itself.
hipError_t launch_mag_sweep(hipStream_t s, int kinds, const SweepArgs &a, SweepLaunch L, hipEvent_t e0 = nullptr,
                            hipEvent_t e1 = nullptr);
// Wall correction data (device pointers), markers in the library's internal order.
struct IbArgs {
    int64_t N;
    int M, nband, tm, km;
    const int *tap_cell;   // [tm][M] cells of the taps (padded taps repeat a valid cell)
    const float *tap_w;    // [tm][M] weights D_jk (0 for padding)
    const float *sj;       // [M] diagonal scaling
    const float *wall;     // [3][M] imposed wall values
    const int *band_cell;  // [nband] cells touched by some marker, increasing
    const int *band_mk;    // [km][nband] marker of each gather entry (padding: a valid marker)
    const float *band_w;   // [km][nband] weight of each gather entry (0 for padding)
    float *delta;          // [3][M] Lagrangian corrections
    const void *phi_hi;    // split form: hi part of the field, added in the interpolation (else NULL)
    void *copy;            // float16 copy of the field refreshed at corrected cells (else NULL)
    float copy_inv;        // 1 / scale of that copy
    // Line-structured walls (ring != 0): every marker sits on an integer x plane and the markers
    // form lines, one marker per x plane at each (y, z) position, internal index j = line * nx + x,
    // n_x a multiple of 64. Taps and gather entries then repeat along x and are read from
    // per-line and per-band-row tables (wave-uniform); band cell e = row * nx + x.
    int ring, nx, kmr;
    const int *ring_tap;   // [lines][tm] tap offsets nx (y + ny z) (padding repeats the first)
    const float *ring_tw;  // [lines][tm] tap weights (0 for padding)
    const int *row_off;    // [rows] offset nx (y + ny z) of each band row, increasing
    const int *row_mk;     // [rows][kmr] line of each gather entry (padding: a valid line)
    const float *row_w;    // [rows][kmr] weight of each gather entry (0 for padding)
};
// Interpolation launch, then spreading launch.
hipError_t launch_ib(hipStream_t s, int kind, void *phi, float scale, float inv_scale, const IbArgs &a);
// b_hi: hi part of b in the split form (else NULL); bext_yz: (y, z) table added to bext, or NULL.
hipError_t launch_lorentz(hipStream_t s, int kind_b, const void *b, const void *b_hi, const float *bext,
                          const float *bext_yz, const DevCtrl *ctrl, float *F, StepConst c);
// u_copy: float16 copy of the new u (u / u_scale) for the split form's sweeps (else NULL).
hipError_t launch_fluid(hipStream_t s, int kinds, const void *rho, const void *u, const float *F,
                        void *rho_o, void *u_o, void *u_copy, StepConst c);
hipError_t launch_flow_partial(hipStream_t s, int kind_u, const void *u, double *part, StepConst c);
// Lorentz force and fluid update in one launch (float32 single boxes; k_lorentz_fluid).
struct LfArgs {
    const float *rho, *u, *b;     // state before the fluid update (b after the magnetic iteration)
    const float *bext, *bext_yz;  // B_ext tables (bext_yz NULL unless six magnets)
    const DevCtrl *ctrl;
    float *rho_o, *u_o;           // new rho - 1 and u* (before the u wall correction)
    StepConst c;
    int tiles_x, tiles_y, zchunk, nblocks;  // filled in by the launcher
};
hipError_t launch_lorentz_fluid(hipStream_t s, const LfArgs &a);
// ring == NULL: the partials only (for launch_residual_final).
hipError_t launch_budget(hipStream_t s, int kinds, const void *rho, const void *u, const void *b,
                         const void *b_hi, const float *bext, const float *bext_yz, DevCtrl *ctrl, double *part,
                         mhd_budget *ring, StepConst c);
// -------------------------------------------------------------------------------------------
// Batched launches: one launch covers the same kernel for many boxes. Each workgroup finds its
// box and its workgroup index within that box in a map of (box, local workgroup) pairs, then
// reads the box's arguments from a device table of PipeStep records and runs the same body as
// the single-box kernel, so every box gets bitwise the result of its own single-box launch.
// -------------------------------------------------------------------------------------------
struct PipeStep {
    SweepArgs sw[3];          // sweep of round 0, of an odd round, of an even round >= 2 (the b
                              // buffers swap every round; round 0 also re-splits the split form)
    IbArgs ib[3];             // wall correction of b after an even round, after an odd round; of u
    void *phi[3];             // field corrected by ib[i]
    float scale[3], inv_scale[3];
    const void *b_last;       // b after the box's last sweep (Lorentz input)
    const void *b_hi;         // split form: hi part of b during and after the sweeps (else NULL)
    const float *bext_yz;     // (y, z) table of B_ext (six magnets), else NULL
    void *u_copy;             // split form: float16 copy of u written by the fluid kernel (else NULL)
    const float *bext;
    DevCtrl *ctrl;
    float *F;
    const void *rho, *u;      // fluid input
    void *rho_o, *u_o;        // fluid output (input of the flow-rate sum)
    double *flow_part;
    double inv_count;
    StepConst c;
};
static_assert(sizeof(PipeStep) % 8 == 0, "PipeStep is copied as an array");
struct BlockMap {             // (box, workgroup within the box) of workgroup i of a batched launch
    int pipe, local;
};
hipError_t launch_ctrl_begin_batch(hipStream_t s, const PipeStep *tab, int n);
hipError_t launch_step_end_batch(hipStream_t s, const PipeStep *tab, int n);
hipError_t launch_mag_sweep_batch(hipStream_t s, int kinds, SweepLaunch L, const PipeStep *tab, const BlockMap *map,
                                  int parity, int nblocks, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_ib_interp_batch(hipStream_t s, int kind, const PipeStep *tab, const BlockMap *map, int which,
                                  int nblocks);
hipError_t launch_ib_spread_batch(hipStream_t s, int kind, const PipeStep *tab, const BlockMap *map, int which,
                                  int nblocks);
// q27: the lattice of every box of the batch (a batch holds one lattice)
hipError_t launch_lorentz_batch(hipStream_t s, int kind_b, const PipeStep *tab, const BlockMap *map, int nblocks,
                                bool q27);
hipError_t launch_fluid_batch(hipStream_t s, int kinds, const PipeStep *tab, const BlockMap *map, int nblocks,
                              bool q27);
hipError_t launch_flow_partial_batch(hipStream_t s, int kind_u, const PipeStep *tab, int n);
// Workgroups per box of the cell-wise kernels and of the wall-correction launches.
constexpr int kCellThreads = 256;
constexpr int kIbThreads = 256;

// float32 staging <-> storage kind (round to nearest even on the way in).
hipError_t launch_store_kind(hipStream_t s, int kind, const float *src, void *dst, int64_t n);
hipError_t launch_load_kind(hipStream_t s, int kind, const void *src, float *dst, int64_t n);
// float32 staging -> float16 hi = fp16(v), lo = fp16(v - hi) (values already divided by the scale).
hipError_t launch_store_split(hipStream_t s, const float *src, void *hi, void *lo, int64_t n);
hipError_t launch_reset_records(hipStream_t s, DevCtrl *ctrl);
// Residual sum of budget partials (slot 13) -> out = sqrt(sum / n_omega) (one workgroup).
hipError_t launch_residual_final(hipStream_t s, const double *part, double *out);

// Stepping with the step scratch outside the workspace (mhd_runtime.cpp; used by the
// allocation-free entry point in mhd_noalloc.hip).
mhd_status step_checks(mhd_sim *s, int64_t n_steps);      // the argument checks of mhd_step
size_t step_scratch_bytes(const mhd_sim *s);              // scratch one step of this box needs
// n_steps steps with direct launches, the step kernels' scratch at dev_scratch (device memory of
// at least step_scratch_bytes(s) bytes, 256-byte aligned)
mhd_status step_in_scratch(mhd_sim *s, int64_t n_steps, int32_t budget_every, void *dev_scratch);
mhd_status report_error(mhd_status st, const char *msg);  // sets mhd_last_error
int sim_device(const mhd_sim *s);

// Packs the three storage kinds (rho, u, b) into one dispatch code.
inline int pack_kinds(int r, int u, int b) { return r | (u << 4) | (b << 8); }

}  // namespace mhd
