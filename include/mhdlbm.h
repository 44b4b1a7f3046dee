/*
 * mhdlbm — C ABI of the MI355X (gfx950) single-step simplified lattice Boltzmann solver for
 * quasi-static MHD pipe flow with an explicit immersed-boundary wall
 * (Tavares, Magacho, Moriconi, Loureiro, arXiv:2211.09370).
 *
 * Problem statement followed by the calls (Sec. 4 and Sec. 5): a box of nx*ny*nz lattice cells,
 * periodic on every face, holds a conducting fluid driven along x by a body force G(t) (the
 * pressure gradient, dp/dx = -G, Sec. 4 variable-force form G(t) = G0 + G1 cos(2 pi t / T)).
 * An imposed field B_ext (uniform along y, or a tanh fringe along y that varies with x) acts on
 * it; the induced field b is iterated in the quasi-static limit (Sec. 5.7). An insulating pipe
 * wall is represented by Lagrangian markers at which u = u_wall and b = b_wall (default 0) are
 * imposed with the explicit immersed boundary of Sec. 5.3 - 5.6.
 *
 * Units are lattice units (dx = dt = 1, Sec. 4). Every field crosses the ABI as float64,
 * component-major, x fastest: element (a, x, y, z) of a vector field is at
 * a*nx*ny*nz + x + nx*(y + ny*z).
 *
 * Errors: every call returns an mhd_status; on failure mhd_last_error() gives a message
 * (thread-local, valid until the next call on the same thread). No call aborts the process.
 * Threading: one mhd_sim must not be used by two threads at once.
 */
#ifndef MHDLBM_H
#define MHDLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mhd_status;
#define MHD_OK 0
#define MHD_ERR_INVALID_ARG (-1) /* argument out of range or inconsistent                   */
#define MHD_ERR_OOM (-2)         /* workspace too small / host allocation failed            */
#define MHD_ERR_HIP (-3)         /* a HIP runtime call failed (message names it)            */
#define MHD_ERR_UNSTABLE (-4)    /* non-finite state or |u| >= c_s found by the fluid update
                                    of any step or by a budget pass (c_s = 1/sqrt(3);
                                    6 nu / sqrt(3) on the macroscopic fluid branch)         */
#define MHD_ERR_STATE (-5)       /* call out of order (e.g. step before params/markers)     */
#define MHD_ERR_UNSUPPORTED (-6) /* valid request outside this build (e.g. gamma != 1 with
                                    tau >= 1)                                               */

/* Storage kind of a field in device memory. Arithmetic is always float32. 16-bit kinds store
 * offsets: rho as rho - 1, u as u / u_scale, b as b / b_scale.
 * MHD_STORE_F16_SPLIT (b only, with rho and u float32): b = (hi + lo) b_scale with two float16
 * arrays; hi is re-quantised once per fluid step (first sweep) and the sweeps update lo, so the
 * 16-bit rounding is relative to the change of b rather than to b. The sweeps then read a float16
 * copy of u (u / u_scale) that the fluid step and its wall correction keep current.
 * Built mixes (rho, u, b): all F32; F16, F16, F16; F16, BF16, F16; all BF16; F32, F32, F16_SPLIT. */
typedef enum { MHD_STORE_F32 = 0, MHD_STORE_F16 = 1, MHD_STORE_BF16 = 2, MHD_STORE_F16_SPLIT = 3 } mhd_storage;

typedef struct {
    int32_t nx, ny, nz;    /* box size in cells; nx, ny, nz >= 1                         */
    int32_t rho_storage;   /* mhd_storage of the density offset rho - 1                  */
    int32_t u_storage;     /* mhd_storage of the velocity                               */
    int32_t b_storage;     /* mhd_storage of the induced field                          */
    double u_scale;        /* velocity scale of 16-bit storage and of the split form's
                              float16 copy of u (> 0; else ignored)                    */
    double b_scale;        /* induced-field scale of 16-bit storage (> 0; ignored for F32) */
} mhd_grid_desc;

typedef enum {
    MHD_BEXT_NONE = 0,
    MHD_BEXT_UNIFORM_Y = 1,     /* B_ext = (0, B0, 0)                                    */
    MHD_BEXT_TANH_FRINGE_Y = 2, /* B_ext = (0, B0 (1 + tanh((x - fringe_x0)/fringe_w))/2, 0) */
    MHD_BEXT_SIX_MAGNETS = 3    /* six magnets with alternating poles on a hexagon around the
                                   axis (yc, zc) (Sec. 6): one magnet's field in its own frame is
                                   B_y' = 2 [atan((y'-L)/z') - atan((y'+L)/z')],
                                   B_z' = log(((y'+L)^2 + z'^2) / ((y'-L)^2 + z'^2)) (a strip of
                                   half-width L on z' = 0); magnet m at angle 60 m degrees,
                                   distance magnet_distance, strip tangential, z' radial outwards,
                                   polarity (-1)^m; scaled so |B_ext| = B0 at (yc + R, zc), R =
                                   avg_radius. Independent of x.                             */
} mhd_bext_kind;

/* Physical parameters (lattice units). */
typedef struct {
    double nu;            /* kinematic viscosity (> 0). tau = 3 nu / gamma + 1/2 selects the
                             fluid update: tau < 1, the single-step predictor (Sec. 3.3, 5.1);
                             tau >= 1 (gamma = 1 only), the macroscopic tau = 1 update with
                             particle speed c = 6 nu (Sec. 5.7), one step then advancing the
                             time by 1 / (6 nu) (forces act over that step)                  */
    double eta;           /* magnetic resistivity (> 0); particle speed of the b iteration
                             c = 6 eta, kappa = 1/(2 eta) (Sec. 5.7)                      */
    int32_t n_mag;        /* magnetic sweeps per fluid step (>= 1), usually
                             min(ceil(6 eta), 270) (Sec. 5.7 iteration count and cap)       */
    int32_t bext_kind;    /* mhd_bext_kind                                                 */
    double lambda_u;      /* viscosity ratio of the u correction (Sec. 5.5); <= 0 -> 1      */
    double lambda_b;      /* resistivity ratio of the b correction (Sec. 5.6); <= 0 -> 6 eta
                             (reference resistivity 1/6)                                   */
    double G0, G1, period;/* G(t) = G0 + G1 cos(2 pi t / period); period <= 0 -> G = G0     */
    double B0;            /* imposed field amplitude                                       */
    double fringe_x0, fringe_w; /* tanh fringe centre and width (cells), fringe_w > 0       */
    double yc, zc;        /* pipe axis position in the cross-section (cells)               */
    double avg_radius;    /* pipe radius R used by the budgets (r < R - 2) and flow rate   */
    int32_t flow_control; /* 1: integral control of G towards u_bulk_target               */
    int32_t lattice;      /* velocity set of both iterations: 0 or 19 -> D3Q19; 27 -> D3Q27, the
                             paper's own set (Table I; weights 8/27, 2/27, 1/54, 1/216), with
                             float32 or split storage only (UNSUPPORTED otherwise)            */
    double u_bulk_target; /* target bulk velocity over r <= R                               */
    double k_c;           /* control gain: G += k_c (8 nu / R^2) (target - U_b) per step    */
    double alpha;         /* accelerated magnetic iteration (Sec. 5.8, eq. "magnetic field
                             quasi-static acelerated"): rest population (w_0 - 1 + alpha) b,
                             gathered sum divided by alpha, i.e. b' = b + (S(b) - b) / alpha
                             with S the plain sweep; same fixed point, slow modes converge
                             1/alpha times faster. 0 or 1: plain sweep. Must be >= 4/9 on
                             D3Q19, >= 13/27 on D3Q27 (the averaging symbol's minimum is 1/9,
                             resp. 1/27; smaller alpha diverges).                          */
    double magnet_half_width; /* six magnets: L; <= 0 -> avg_radius / 6 (Sec. 6)            */
    double magnet_distance;   /* six magnets: distance of the strip centres from the axis;
                                 <= 0 -> distance of the farthest cell of the box from the axis
                                 + L + 1 (no strip reaches into the box)                      */
    double gamma;         /* time-step rescaling of the fluid update (Sec. 7): dt -> dt / gamma,
                             c_i -> gamma c_i. The quadratic part of f^eq is divided by gamma,
                             tau = 3 nu / gamma + 1/2, the GZS populations take their rescaled
                             form and the explicit force term is F / gamma, so a steady state
                             does not depend on gamma and a transient takes gamma times as many
                             steps. <= 0 or 1: no rescaling. The magnetic iteration is unchanged
                             (quasi-static: it has no time step).                             */
    double omega_radius;  /* radius of the budget region Omega = {(y-yc)^2 + (z-zc)^2 <
                             omega_radius^2}; <= 0 -> avg_radius - 2 (inside the band the wall
                             kernel touches). avg_radius selects the whole conductor, where the
                             steady power balance P_in = -P_nu + D_eta holds (Sec. 4).        */
} mhd_params;

typedef enum { MHD_FIELD_RHO = 0, MHD_FIELD_U = 1, MHD_FIELD_B_INDUCED = 2 } mhd_field;

/* One budget record (Sec. 4 energy balance): averages over Omega = {(y-yc)^2 + (z-zc)^2 <
 * R_omega^2} (R_omega = omega_radius, default R - 2) of E_k = <rho |u|^2 / 2>, E_m = <|B|^2 / 2> (B = B_ext + b), E_b = <|b|^2 / 2>,
 * P_in = G <u_x>, P_p = -<u . grad(rho/3)>, P_nu = nu <u . lap u>, P_L = <u . (J x B)>,
 * M_eta = eta <B . lap b>, M_adv = -<B . div(u B - B u)>, joule = eta <|J|^2>; plus
 * mass = sum of rho over the box, Q = (1/nx) sum over r <= R of u_x, u_max = max |u|.
 * Derivatives are the D3Q19 isotropic differences; all sums are float64 in a fixed order. */
typedef struct {
    int64_t step;   /* steps completed when the record was taken                          */
    double G;       /* body force used by that step                                       */
    double E_k, E_m, E_b, P_in, P_p, P_nu, P_L, M_eta, M_adv, joule, mass, Q, u_max;
    double n_omega; /* number of cells in Omega                                            */
    double res_mag; /* induction residual (Sec. 5.8 eq. "Error l2 decay"): root mean square
                       over Omega of |eta lap b - div(u B - B u)|; the paper normalises it by
                       its value at the first iteration                                      */
    double D_eta;   /* Joule dissipation in lattice Dirichlet form, -eta <b . lap b> (equal to
                       eta <|J|^2> for a divergence-free b vanishing on the boundary of Omega;
                       with -P_nu, the viscous dissipation in the same form, a steady state over
                       the conductor satisfies P_in = -P_nu + D_eta and -P_L = D_eta)        */
} mhd_budget;

typedef struct mhd_sim mhd_sim;

/* Thread-local message of the last failing call ("" if none). */
const char *mhd_last_error(void);

/* Bytes of device workspace needed for a box g with at most n_markers markers
 * (host-only; no GPU needed). */
mhd_status mhd_workspace_size(const mhd_grid_desc *g, int64_t n_markers, size_t *bytes);

/* Create a solver on the current HIP device.
 * dev_workspace: device memory of at least mhd_workspace_size(g, n_markers) bytes, 256-byte
 *   aligned, owned by the caller and kept alive until mhd_destroy.
 * hip_stream: the hipStream_t every kernel and copy is issued on (NULL = default stream).
 * Fields start at rho = 1, u = 0, b = 0, t = 0. */
mhd_status mhd_create(const mhd_grid_desc *g, int64_t n_markers, void *dev_workspace, size_t bytes,
                      void *hip_stream, mhd_sim **out);

/* Wall markers X_j (host, SoA: x[0..M), y[0..M), z[0..M)) and the imposed wall values
 * u_wall, b_wall (host, 3*M component-major, NULL -> 0). Copied; caller keeps ownership.
 * Each coordinate must lie in [0, n) of its axis (the stencil wraps periodically).
 * Computes the Lagrange taps (Sec. 5.2), the row sums d_j of D D^T (Sec. 5.3) and the
 * gather lists of the spreading step. M = 0 removes the wall. A wall made of lines (every
 * marker on an integer x plane and, at each (y, z) position, one marker on every x plane, as
 * the rings of a straight pipe) with n_x a multiple of 64 is also stored as per-line and
 * per-band-row tables, which the corrections then read (the same taps and entries in the
 * same order, so the same results). The environment variable MHD_IB_RING, read here, selects:
 * 0 = general tables only, 1 (default) = line tables where the wall allows, 2 = line tables
 * required (UNSUPPORTED otherwise). */
mhd_status mhd_set_markers(mhd_sim *s, const double *xyz, int64_t M, const double *u_wall,
                           const double *b_wall);

/* Parameters (copied). INVALID_ARG if nu <= 0, eta <= 0, n_mag < 1, a fringe width <= 0,
 * 0 < alpha below its lattice bound, or (with markers set) 1 + d_j (lambda - 1) <= 0 for some
 * marker (the scaling of Sec. 5.5 / 5.6 would be singular or negative). UNSUPPORTED if
 * tau = 3 nu / gamma + 1/2 >= 1 with gamma != 1 (the macroscopic branch has no rescaling). */
mhd_status mhd_set_params(mhd_sim *s, const mhd_params *p);

/* Copy a field in / out (host float64, layout above; rho has 1 component, u and b 3).
 * Synchronous with respect to the host buffer. mhd_get_field also reports a deferred
 * MHD_ERR_UNSTABLE: set by the fluid update of any step whose new velocity at some cell is
 * non-finite or has |u| >= c_s, or by a budget pass, whatever budget_every is (the data is
 * still copied; the flag stays set for the life of the solver). */
mhd_status mhd_set_field(mhd_sim *s, mhd_field f, const double *host);
mhd_status mhd_get_field(mhd_sim *s, mhd_field f, double *host);

/* Step counter and current body force (checkpoint / resume). */
mhd_status mhd_get_time(mhd_sim *s, int64_t *t, double *G);
mhd_status mhd_set_time(mhd_sim *s, int64_t t, double G);

/* Advance n_steps fluid steps (each: n_mag magnetic sweeps with the b correction after each,
 * Lorentz force, fluid predictor, u correction). Asynchronous on the stream: returns after
 * the launches. If budget_every > 0 a budget record is taken after every step whose new step
 * count is a multiple of budget_every. On a caller stream (hip_stream != NULL at mhd_create)
 * with graphs enabled and profiling off, the first step from each state of the double buffers
 * is captured into a HIP graph (stream capture, relaxed mode: do not enqueue other work on
 * that stream from another thread meanwhile) and every step is one graph launch; the graphs
 * are dropped when parameters, markers or tiles change. Results are the same as with direct
 * launches. */
mhd_status mhd_step(mhd_sim *s, int64_t n_steps, int32_t budget_every);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): mhd_step with the scratch of its kernels (Lorentz
 * force, wall corrections, flow-rate and budget partials) in a static device array of the library
 * (32 MiB per GPU, held until the process ends) instead of the solver's workspace. Same kernels
 * and launch order as mhd_step, issued directly (no graph), so the results are the same bit for
 * bit; the caller still provides the fields (the solver's workspace) and the stream. No call
 * allocates, frees or clears memory; every scratch value is written before it is read within a
 * step. INVALID_ARG if the box needs more than the array holds (about 2.7 M cells); the other
 * errors as mhd_step. All calls on one GPU share that GPU's array: calls whose work overlaps on
 * the GPU (two solvers on different streams, or another thread) race on it, so serialise them. */
mhd_status mhd_step_noalloc(mhd_sim *s, int64_t n_steps, int32_t budget_every);

/* Graph replay of mhd_step (performance only): enable = 1 (default) or 0 (direct launches). */
mhd_status mhd_set_graph(mhd_sim *s, int32_t enable);

/* Synchronise the stream and move the budget records taken since the last call (oldest first,
 * at most cap) to out. Returns MHD_ERR_UNSTABLE if a fluid step or a record found non-finite
 * values or |u| >= c_s (the records are still returned). */
mhd_status mhd_get_budgets(mhd_sim *s, mhd_budget *out, int64_t cap, int64_t *n_out);

/* Take one budget record of the current state now (asynchronous). */
mhd_status mhd_record_budget(mhd_sim *s);

/* Induction residual along the magnetic iteration (Sec. 5.8, eq. "Error l2 decay"), for choosing
 * n_mag: from the current state, runs n_sweeps (1 .. 4096) magnetic sweeps, each followed by the
 * b wall correction, with u and the step counter held, and writes to res_out[k] (host, n_sweeps
 * doubles) the residual res_mag (see mhd_budget) after sweep k + 1. The paper normalises the
 * curve by its first value and takes the smallest count whose damping is sufficient. The
 * induced field is restored afterwards, so the state is unchanged. Synchronous. */
mhd_status mhd_mag_residual_curve(mhd_sim *s, int32_t n_sweeps, double *res_out);

/* Effective number of magnetic sweeps (Sec. 5.8: the count at which the iteration has damped
 * enough, instead of a non-local residual every step): from the current state, the residual curve
 * above over n_max sweeps (1 .. 4096), and *n_out = the smallest n whose residual is at most
 * tol (0 < tol < 1) times the residual after the first sweep, or n_max if none is. The state is
 * unchanged. apply = 1 also makes it the solver's n_mag (as mhd_set_params would). Synchronous. */
mhd_status mhd_choose_n_mag(mhd_sim *s, double tol, int32_t n_max, int32_t apply, int32_t *n_out);

/* Kernel timing with HIP events on the solver's stream: when enabled, mhd_step brackets every
 * launch of the kernels with events; mhd_kernel_stats synchronises and returns the number of
 * timed launches and their summed duration for one kernel id, then forgets them. */
typedef enum {
    MHD_K_MAG_SWEEP = 0, /* magnetic sweep                                              */
    MHD_K_IB = 1,        /* wall correction of b or u (one launch, two for huge groups)  */
    MHD_K_LORENTZ = 2,
    MHD_K_FLUID = 3,
    MHD_K_BUDGET = 4,
    MHD_K_CONTROL = 5,   /* body force, flow-rate control, step counter                  */
    MHD_K_COUNT = 6
} mhd_kernel_id;
mhd_status mhd_set_profiling(mhd_sim *s, int32_t enable);
mhd_status mhd_kernel_stats(mhd_sim *s, int32_t kernel, int64_t *launches, double *total_ms);

/* Free library host state (events included). Device workspace stays the caller's.
 * STATE for a box of a batch (mhd_batch_destroy frees those). */
mhd_status mhd_destroy(mhd_sim *s);

/* Tile choice of the magnetic sweep (performance only): tiles[0] = x tile (8, 16, 32 or 64
 * cells, 256 work-items per workgroup), tiles[1] = z planes marched per workgroup (>= 1),
 * tiles[2] = 1 for two x cells per lane with 128-cell x tiles (used only when nx is a multiple
 * of 128), tiles[3] = rows per workgroup of that form (4 or 8). Results do not depend on the
 * choice beyond float32 rounding of contracted multiply-adds. Default: the widest x tile the box
 * fills, the paired form when it applies, and the longest z chunk of 64, 32 or 16 planes that
 * leaves 512 workgroups (paired float32 sweep) or 2048 (other forms), else 8; rows 4, or 8 for
 * paired float32 chunks of 32 planes or more when 256 workgroups remain, with the chunk then
 * doubled up to 128 planes while 256 workgroups still remain. */
mhd_status mhd_get_tiles(mhd_sim *s, int32_t tiles[4]);
mhd_status mhd_set_tiles(mhd_sim *s, const int32_t tiles[4]);

/* Autotuner of the sweep tiles of one box: every valid choice (x tile 8-64, the paired form with
 * 4 or 8 rows when nx % 128 == 0, z chunks 4-128 planes) is timed by reps sweeps (default 5 if
 * reps <= 0) of the live fields into the box's other buffer of b, and the fastest is kept. The
 * state is unchanged. Synchronous. STATE before mhd_set_params or on a box of a batch. */
mhd_status mhd_tune(mhd_sim *s, int32_t reps);

/* ---------------------------------------------------------------------------------------------
 * Batched form: many independent pipes (boxes), each with its own size, markers, parameters and
 * number of magnetic sweeps, advanced together. One fluid step of the whole batch is a fixed
 * sequence of launches, each covering every box that takes part in it: sweep round r runs on
 * the boxes with n_mag > r, followed by their b wall correction; then Lorentz, fluid and u wall
 * correction run on all boxes. With graphs enabled (default) that sequence is captured once in
 * a HIP graph per state of the boxes' double buffers and replayed, one graph launch per step.
 * Every box evolves bitwise as a single box with the same tile choice would.
 * ------------------------------------------------------------------------------------------- */
typedef struct mhd_batch mhd_batch;

typedef struct {
    mhd_grid_desc grid;   /* box of this pipe; all pipes of a batch share the storage kinds   */
    int64_t n_markers;    /* marker capacity of this pipe                                      */
} mhd_pipe_desc;

/* Bytes of device workspace for the batch (host-only). */
mhd_status mhd_batch_workspace_size(const mhd_pipe_desc *pipes, int32_t n, size_t *bytes);

/* Create a batch of n >= 1 pipes on the current device; workspace and stream rules as for
 * mhd_create. A stream of NULL disables graphs (the NULL stream cannot be captured). */
mhd_status mhd_batch_create(const mhd_pipe_desc *pipes, int32_t n, void *dev_workspace, size_t bytes,
                            void *hip_stream, mhd_batch **out);

/* Handle of pipe i, owned by the batch. mhd_set_markers, mhd_set_params, mhd_set_field,
 * mhd_get_field, mhd_get_time, mhd_set_time, mhd_record_budget, mhd_get_budgets and the tile
 * calls work on it as on a single box; mhd_step and mhd_destroy return STATE. */
mhd_status mhd_batch_pipe(mhd_batch *b, int32_t i, mhd_sim **out);

/* Autotuner of the sweep tiles (mhd_get_tiles). Pipes are grouped by nx; for each group in
 * turn, every valid tile choice is tried with the other groups fixed by timing reps (default 5
 * if reps <= 0) batched sweep rounds over the whole batch on the live fields, and the fastest
 * is kept; two passes, starting from the current choice. The timed sweeps write only the
 * scratch copy of b, so the state is unchanged. Synchronous. */
mhd_status mhd_batch_tune(mhd_batch *b, int32_t reps);

/* Advance every pipe by n_steps fluid steps (asynchronous, like mhd_step). If budget_every > 0,
 * each pipe records a budget after every step whose new step count is a multiple of it. STATE
 * if a pipe has no parameters. */
mhd_status mhd_batch_step(mhd_batch *b, int64_t n_steps, int32_t budget_every);

/* 1 (default): replay captured graphs; 0: issue the launches directly. */
mhd_status mhd_batch_set_graph(mhd_batch *b, int32_t enable);

/* Kernel timing as mhd_set_profiling / mhd_kernel_stats, per batched launch (graphs are
 * bypassed while profiling is on). */
mhd_status mhd_batch_set_profiling(mhd_batch *b, int32_t enable);
mhd_status mhd_batch_kernel_stats(mhd_batch *b, int32_t kernel, int64_t *launches, double *total_ms);

/* Free the batch, its pipes and its graphs. Device workspace stays the caller's. */
mhd_status mhd_batch_destroy(mhd_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* MHDLBM_H */
