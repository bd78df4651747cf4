/*
 * csph.h -- C ABI of the MI355X (gfx950) CSPH-TVD solver for the coupled
 * Saint-Venant shallow-water and Exner bed-evolution equations of Khrapov &
 * Khoperskov, "Application of GPUs for self-consistent modelling of shallow
 * water dynamics and sediment transport", Lobachevskii J. Math. 41(8) (2020).
 *
 * The library mirrors the paper's Section 3 software layout: the caller is the
 * control block (Main: loads the bed, soil and friction fields and the initial
 * state), the library is the computing block (Solver: the step kernels on the
 * GPU), and field/sum readback replaces the Save/Screen blocks, so the host
 * and the device exchange data only when the caller asks.
 *
 * Conventions (every function):
 *  - Return value: 0 (SW_OK) or a negative SW_ERR_* code; sw_last_error(ctx)
 *    gives a text for the last failure on that context.  No C++ exception
 *    crosses this boundary.
 *  - Fields are row-major [ny][nx] float32 arrays, x fastest, SI units
 *    (depth h in m, unit discharges hu, hv in m^2/s, bed elevation b in m).
 *  - ptr_kind SW_PTR_HOST: the pointer is host memory, copied synchronously
 *    and in the context's stream order, through a pinned staging buffer the
 *    library owns (pageable user memory is never handed to a device copy).
 *    SW_PTR_DEVICE: the pointer is device memory on the context's GPU (for
 *    instance a torch tensor's data_ptr()); the copy is ordered on the
 *    context's stream.  The caller keeps ownership of its buffers; the library
 *    owns every device allocation it makes and frees them in sw_destroy.
 *  - Work is ordered on the context's HIP stream (the stream passed to
 *    sw_create, or one the library creates).  sw_get_fields and sw_get_sums
 *    synchronise that stream.
 *  - A context is used by one host thread at a time.
 *  - Sides are indexed W=0 (x = 0), E=1 (x = max), S=2 (y = 0), N=3 (y = max).
 */
#ifndef CSPH_H
#define CSPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SW_OK 0
#define SW_ERR_ARG (-1)          /* bad argument (size, pointer, range) */
#define SW_ERR_HIP (-2)          /* a HIP runtime call failed */
#define SW_ERR_NONFINITE (-3)    /* a NaN/Inf appeared in the state */
#define SW_ERR_DT_UNDERFLOW (-4) /* the Eq. 7 step fell below dt_min */
#define SW_ERR_STATE (-5)        /* call out of order (advance before set_state, ...) */
#define SW_ERR_CFL (-6)          /* a fixed dt exceeds the Eq. 7 step */

#define SW_BC_WALL 0 /* reflective wall: ghost cell mirrors the normal velocity */
#define SW_BC_OPEN 1 /* zero-gradient: ghost cell copies the boundary cell */

#define SW_SED_NONE 0  /* no bed evolution */
#define SW_SED_GRASS 1 /* Grass law J0 = A_G |v|^m_exp v (Eq. 3) */
#define SW_SED_EQ4 2   /* J0 = A |v|^4 v with A = 0.05 nM^3 / ((s-1) sqrt(g h) d50) (Eqs. 3-4) */

#define SW_PTR_HOST 0
#define SW_PTR_DEVICE 1

/* TVD limiter of the Euler stage (Section 3 names TVD limiters without fixing
 * one): minmod (default), MC (monotonised central, van Leer 1977), superbee
 * (Roe 1985). */
#define SW_LIM_MINMOD 0
#define SW_LIM_MC 1
#define SW_LIM_SUPERBEE 2

/* HLL wave-speed estimate of the Euler stage: Davis (default), or the
 * two-rarefaction estimate of Toro (star celerity (cL + cR)/2 + (uL - uR)/4,
 * star velocity (uL + uR)/2 + cL - cR; SL = min(uL - cL, u* - c*), SR =
 * max(uR + cR, u* + c*)). */
#define SW_HLL_DAVIS 0
#define SW_HLL_TWO_RAREFACTION 1

/* sw_params.flags */
#define SW_FLAG_HGS 1u        /* skip dry tiles (the hierarchical grid system, Section 3) */
#define SW_FLAG_UNFUSED 2u    /* run the unfused kernel sequence (faces, then update) */
#define SW_FLAG_NO_GRAPH 4u   /* launch kernels one by one instead of replaying a HIP graph */
/* Second-order Lagrangian force (the K2/K5 pressure and bed-slope force of
 * Eq. 6 on hydrostatic faces of states reconstructed with the TVD limiter,
 * plus Audusse et al.'s centred bed-slope term; a reading: the paper names
 * TVD reconstruction for the Euler stage only).  Built into the strip
 * kernels: with it, LDS tile shapes (sw_set_tile_shape) and SW_FLAG_UNFUSED
 * are SW_ERR_ARG, the autotuners try strip shapes only, and an ensemble's
 * members must all have it or all lack it. */
#define SW_FLAG_FORCE2 8u

typedef struct sw_ctx sw_ctx;

/* Uniform grid: nx * ny square cells of side dx (the cell size h of Eq. 7). */
typedef struct {
    int32_t nx, ny;
    double dx;
    int32_t bc[4]; /* SW_BC_* per side W, E, S, N */
} sw_grid;

/* Model constants; sw_default_params fills the defaults named here. */
typedef struct {
    double g;       /* gravity, 9.81 m/s^2 */
    double cfl;     /* Courant number K of Eq. 7, 0.3 */
    double eps_dry; /* desingularisation depth of the velocity, 1e-5 m */
    double h_sed;   /* no bedload at or below this depth, 1e-2 m */
    double dt_max;  /* cap on the Eq. 7 step, 1 s */
    double dt_min;  /* smaller Eq. 7 steps are an error, 1e-9 s */
    double s_rel;   /* s = rho_s / rho of Eq. 4, 2.65 */
    double C_J;     /* bed-slope coefficient of Eq. 2, 2.0 */
    double C_Sh;    /* Shamov coefficient of Eq. 5, 5.0 */
    double A_G;     /* Grass coefficient of Eq. 3, 1e-3 */
    double m_exp;   /* Grass exponent of Eq. 3, 2 */
    int32_t sed_law;/* SW_SED_*, default SW_SED_EQ4 */
    uint32_t flags; /* SW_FLAG_*, default SW_FLAG_HGS */
    int32_t limiter;    /* SW_LIM_*, default SW_LIM_MINMOD */
    int32_t hll_speeds; /* SW_HLL_*, default SW_HLL_DAVIS */
} sw_params;

/* Global diagnostics, all accumulated in FP64 on the device. */
typedef struct {
    double t;                  /* model time */
    double last_dt;            /* the last step taken */
    double water_volume;       /* sum h dx^2 */
    double sediment_volume;    /* sum (1 - psi) b dx^2 (the quantity Eq. 1 conserves) */
    double water_boundary_out; /* accumulated outward boundary water volume */
    double water_source_in;    /* accumulated inflow volume */
    double sed_boundary_out;   /* accumulated outward boundary sediment volume */
    double sed_source_in;      /* accumulated (q_b^+ - q_b^-) dx^2 dt */
    double vp, vs, D;          /* Eq. 7 maxima at the start of the last step (sw_step_bound
                                  takes them over the current fields) */
    int64_t step;              /* step counter */
    int64_t wet_cells;         /* cells with h > 0 */
    int64_t active_tiles;      /* tiles the next step will not skip */
    int64_t cells_lagrange;    /* cells the Lagrangian-stage kernel processed since set_state */
    int64_t cells_euler;       /* cells the Euler-stage kernel processed since set_state */
    int32_t binding_term;      /* Eq. 7 term that set last_dt: 0 h/(2vp), 1 h/vs, 2 h^2/(2D), 3 dt_max, 4 fixed */
    int32_t error;             /* sticky device error (SW_ERR_*), 0 if none */
    int64_t graph_builds;      /* step graphs captured so far: a new state, bed or time
                                  keeps them; soil, sources, forcing, tile shape or a new
                                  fixed dt rebuild them at the next advance */
    double water_rain_in;      /* accumulated rainfall volume */
    double water_absorbed;     /* accumulated volume absorbed (infiltrated) */
} sw_sums;

/* Fill *p with the defaults listed in sw_params. */
void sw_default_params(sw_params *p);

/* Create a solver for `grid`.  hip_stream: a hipStream_t to order all work on
 * (for instance torch.cuda.current_stream().cuda_stream), or NULL to let the
 * library create its own.  The state is all zero until set.  Size limit: a
 * row is padded to a multiple of 64 cells (the pitch), and pitch * ny must
 * stay below 2^30 cells (each field plane under 4 GiB), e.g. up to 32768 x
 * 32767; larger grids, nx or ny < 1 or dx <= 0 are SW_ERR_ARG. */
int sw_create(const sw_grid *grid, const sw_params *params, void *hip_stream, sw_ctx **out);
int sw_destroy(sw_ctx *ctx);

/* Bed elevation b(x, y) (the digital elevation model of Main, Section 3). */
int sw_set_bed(sw_ctx *ctx, const float *b, int ptr_kind);

/* Soil: Manning coefficient nM, median grain size d50 (m) and porosity psi
 * (Eqs. 1, 4, 5, friction in f of Eq. 6).  Each is a per-cell array, or NULL
 * to use the scalar that follows it.  Porosity must lie in [0, 1). */
int sw_set_soil(sw_ctx *ctx, const float *manning, float manning_scalar, const float *d50,
                float d50_scalar, const float *psi, float psi_scalar, int ptr_kind);

/* Initial water depth and unit discharges.  Negative depth is SW_ERR_ARG;
 * the discharge of a cell with zero depth is set to zero.  Resets the step
 * counter, the accumulated balances and any sticky error. */
int sw_set_state(sw_ctx *ctx, const float *h, const float *hu, const float *hv, int ptr_kind);

/* Volumetric inflow (the water source sigma of Eq. 6): n cells (flat
 * indices j*nx+i, host array) with weights (host array, normalised to sum 1
 * by the library) receive Q(t) = q_base + q_peak exp(-(t - t_peak)^2 /
 * (2 t_sigma^2)) m^3/s, evaluated at mid-step; no momentum is added.  n = 0
 * removes the inflow. */
int sw_set_inflow(sw_ctx *ctx, const int32_t *cell_idx, const float *weight, int32_t n,
                  double q_base, double q_peak, double t_peak, double t_sigma);

/* Bed sources q_b^+ (deposition) and q_b^- (erosion drain) of Eq. 1, m/s,
 * per cell; either may be NULL (zero). */
int sw_set_sed_sources(sw_ctx *ctx, const float *qb_plus, const float *qb_minus, int ptr_kind);

/* Forcing named by Eq. 6 without a formula (the water sources sigma and the
 * force f; the Main block's absorption map beta(x, y), Section 3):
 *  - rain: rainfall rate (m/s) on every cell, adding depth without momentum
 *    (with rain > 0 no tile is skipped);
 *  - beta (per-cell array, or NULL for beta_scalar): absorption coefficient
 *    (1/s); dH/dt = -beta H taken implicitly each step (depth and momentum
 *    divided by 1 + beta dt, so the absorbed water leaves with its velocity);
 *  - coriolis: f_c = 2 Omega sin(latitude) (1/s), force f_c (hv, -hu);
 *  - wind_x, wind_y (m/s) and wind_coef C_w = (rho_air / rho_water) C_D:
 *    stress C_w |W| W on water, scaled by min(1, h / h_sed) on thinner layers.
 * Forces enter the predictor at t_n and the corrector at t_{n+1/2}.  All zero
 * (the default) is the plain model.  sw_sums reports water_rain_in and
 * water_absorbed.  Negative or non-finite rain, beta or wind_coef, or
 * non-finite Coriolis and wind values are SW_ERR_ARG. */
int sw_set_forcing(sw_ctx *ctx, double rain, const float *beta, float beta_scalar, double coriolis,
                   double wind_x, double wind_y, double wind_coef, int ptr_kind);

/* Model time and step counter reported by sw_get_sums (does not touch fields). */
int sw_set_time(sw_ctx *ctx, double t, int64_t step);

/* Replace bed and state with device arrays [ny][nx] (dense rows) and set the
 * model time t and step counter: no copy through the host and no check, for
 * drivers that produce states on the GPU (the caller guarantees finite
 * values, h >= 0 and hu = hv = 0 where h = 0).  The Lagrangian momentum, the
 * balances and any pending device error are cleared, as by sw_set_state.
 * Stream-ordered; SW_ERR_ARG for NULL pointers. */
int sw_replace_state(sw_ctx *ctx, const float *h, const float *hu, const float *hv,
                     const float *b, double t, int64_t step);

/* The grid the context was created with. */
int sw_get_grid(const sw_ctx *ctx, sw_grid *out);

/* The Eq. 7 step bound of the current fields: K min(h / (2 vp), h / vs,
 * h^2 / (2 D)) with the cell size h = dx and the maxima vp, vs, D taken over
 * the fields as the next step's K3 takes them, capped at dt_max.  A fixed step
 * above it raises SW_ERR_CFL.  Synchronises; SW_ERR_STATE before
 * sw_set_state, SW_ERR_NONFINITE if a field is not finite, a pending device
 * error is returned as by sw_get_fields. */
int sw_step_bound(sw_ctx *ctx, double *dt);

/* Step log, the record the Screen block of Section 3 shows while a run goes
 * on: each step's time, step length, Eq. 7 maxima and binding term, and the
 * inflow discharge, written by the device when the step's time step is
 * published, into a ring of the last SW_STEP_LOG steps per context (cleared
 * by a new state: sw_set_state, sw_replace_state, sw_checkpoint_load).
 * sw_get_step_log copies the records of the last min(n, steps since the
 * state was set, SW_STEP_LOG) steps, oldest first, into out[] (host memory,
 * n records) and their number into *count (may be NULL).  Synchronises.  A
 * pending device error does not stop it: the records of the steps before the
 * failing one are returned (the failing step has none); SW_ERR_ARG for n < 0
 * or a NULL out with n > 0. */
#define SW_STEP_LOG 1024
typedef struct {
    int64_t step;     /* the step's index (the step counter before it) */
    double t;         /* model time at its start */
    double dt;        /* its length */
    double vp, vs, D; /* Eq. 7 maxima of the state at its start */
    double inflow;    /* hydrograph discharge Q(t + dt/2), m^3/s (0 without inflow) */
    int32_t binding;  /* Eq. 7 term that set dt, as sw_sums.binding_term */
    int32_t reserved;
} sw_step_record;
int sw_get_step_log(sw_ctx *ctx, int32_t n, sw_step_record *out, int32_t *count);

/* Advance nsteps CSPH-TVD steps (Section 3 kernels K1..K8) with the Eq. 7
 * time step.  Asynchronous: errors raised on the device (SW_ERR_NONFINITE,
 * SW_ERR_DT_UNDERFLOW) stop all later steps and are returned by the next
 * sw_get_fields / sw_get_sums / sw_sync; the fields then hold the state at the
 * start of the failing step. */
int sw_advance(sw_ctx *ctx, int32_t nsteps);

/* Same with a fixed step dt; a step whose Eq. 7 bound is below dt raises
 * SW_ERR_CFL on the device (as above). */
int sw_advance_fixed_dt(sw_ctx *ctx, int32_t nsteps, double dt);

/* Measurement aid: advance nsteps (Eq. 7 step) with one launch per kernel on
 * the context's stream, timing the Lagrangian-stage and Euler-stage kernels;
 * on return avg_ms[0] / avg_ms[1] hold their mean durations.  Strip shapes:
 * each launch records its own start and end time stamps (hipExtLaunchKernel
 * events, the kernel's execution as a kernel trace reports it); LDS tile
 * shapes: HIP events recorded between the launches.  Same kernels and
 * arithmetic as sw_advance (the tiled path); synchronises.  SW_ERR_ARG on the
 * unfused path. */
int sw_advance_profiled(sw_ctx *ctx, int32_t nsteps, double *avg_ms);

/* Tile shape of the hierarchical grid of Section 3 (the blocks whose dry
 * members the HGS skips).  Use tile shape tile_x x tile_y for later steps: 64x8, 64x4, 64x16 or 128x4
 * cells per 256-thread workgroup staged through LDS, or 58x8 (the default),
 * 58x16 or 58x32 cells per wavefront (strips: one lane per column plus a
 * 3-column halo, rows marched in registers).  SW_ERR_ARG for any other shape.
 * Results do not depend on the shape (bit-identical). */
int sw_set_tile_shape(sw_ctx *ctx, int32_t tile_x, int32_t tile_y);

/* Tile-shape autotuner for the tiles of the hierarchical grid of Section 3:
 * from the current state, time nsteps of each tile
 * shape the library has (the seven of sw_set_tile_shape), put
 * the state, time and balances back, and keep the fastest shape for every
 * later step.  All shapes give bit-identical results.  Allocates and frees a
 * copy of the state; synchronises.  *tile_x, *tile_y (may be NULL) receive
 * the chosen shape. */
int sw_autotune(sw_ctx *ctx, int32_t nsteps, int32_t *tile_x, int32_t *tile_y);

/* Wait for queued work; returns the sticky device error, if any (the CPU
 * side of the Solver loop of Section 3 waits for the GPU only here and in
 * the two readbacks below). */
int sw_sync(sw_ctx *ctx);

/* Read the current fields h, hu, hv, b (the state the Save and Screen blocks
 * of Section 3 record; any pointer may be NULL to skip that field).
 * Synchronises the context's stream. */
int sw_get_fields(sw_ctx *ctx, float *h, float *hu, float *hv, float *b, int ptr_kind);

/* FP64 global sums of the current state and the accumulated balances (the
 * water volume and the sediment volume of Eq. 1, the Eq. 7 maxima and the
 * boundary and source balances).  Synchronises the context's stream. */
int sw_get_sums(sw_ctx *ctx, sw_sums *out);

/* Asynchronous Save (the Save and Screen blocks of Section 3 record the state
 * every 100-1000 steps; the paper overlaps that exchange with the computation
 * on CUDA streams).  sw_save_begin queues, on the context's stream after the
 * work already queued, a device copy of the current h, hu, hv, b and control
 * block, and on a second stream of its own the copy of that snapshot into
 * pinned host memory the library owns; it returns at once, so later
 * sw_advance calls run while the copy travels.  sw_save_wait blocks until
 * that copy has arrived and writes it into the caller's host arrays
 * [ny][nx] (any may be NULL), with the model time and step of the snapshot
 * (t, step may be NULL); it returns a device error the snapshot carries.  One
 * save may be in flight at a time (SW_ERR_STATE otherwise, and for a wait
 * without a save).  The first call allocates a device snapshot (4 planes)
 * and a pinned host buffer of the same size. */
int sw_save_begin(sw_ctx *ctx);
int sw_save_wait(sw_ctx *ctx, float *h, float *hu, float *hv, float *b, double *t, int64_t *step);

/* Checkpoint and resume (the Save block of Section 3, for restarts): the
 * whole state a later step depends on -- h, hu, hv, the bed and its residual
 * (the part of the accumulated Exner change the float32 bed has not absorbed
 * yet), the model time and step counter, the accumulated inflow, bed-source
 * and boundary balances -- in one host blob the caller owns.  A context
 * created with the same grid, parameters, soil and sources that loads the
 * blob continues bit for bit as the saved one would have.  Size from
 * sw_checkpoint_size; save synchronises and refuses a context with a pending
 * device error (SW_ERR_STATE); load checks the blob's header and grid
 * (SW_ERR_ARG) and replaces the state, time and balances. */
int sw_checkpoint_size(const sw_ctx *ctx, int64_t *bytes);
int sw_checkpoint_save(sw_ctx *ctx, void *buf, int64_t bytes);
int sw_checkpoint_load(sw_ctx *ctx, const void *buf, int64_t bytes);

/* Text of the last error on ctx (never NULL; "" if none). */
const char *sw_last_error(const sw_ctx *ctx);

/* Allocation-free advance, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It runs the kernels of sw_advance (default 58x8 strip shape,
 * skipping dry tiles if params->flags has SW_FLAG_HGS) on a state the caller
 * owns, with every other buffer taken from one file-scope device array of
 * SW_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  It calls no hipMalloc, hipFree, memset or memcpy:
 * set-up, loading and readback are kernels, all ordered on hip_stream (NULL:
 * the null stream), and nothing synchronises.
 *  - h, hu, hv, b: device arrays [ny][nx] on the current GPU, read as the
 *    state at time t0 and overwritten with the state after nsteps steps (or,
 *    after a device error, the state at the start of the failing step).
 *    Scalar soil manning, d50, psi; no inflow and no bed sources.
 *  - dt_fixed = 0: the Eq. 7 step; dt_fixed > 0: that fixed step (a step
 *    above its Eq. 7 bound raises SW_ERR_CFL on the device).
 *  - t_out (device double, may be NULL): the model time of the returned state.
 *  - err_out (device int32, may be NULL): 0, or the device error
 *    (SW_ERR_NONFINITE, SW_ERR_DT_UNDERFLOW, SW_ERR_CFL, or SW_ERR_ARG for a
 *    negative or non-finite input, in which case no step runs).
 *  - errbuf (host, may be NULL): a message for a non-zero return.
 * Returns SW_ERR_ARG without touching the GPU for bad arguments or a grid
 * whose buffers do not fit the array (about 17 x 4 bytes per padded cell:
 * rows padded to a multiple of 64, up to 1,048,576 padded cells, e.g.
 * 1024 x 1024 or 2048 x 512); SW_ERR_HIP if a launch fails.  Every call on a
 * GPU shares that GPU's array and leaves its contents behind: calls that
 * overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller.  The results are bit-identical to sw_create +
 * sw_set_bed/soil/state + sw_set_time(t0) + sw_advance on the same inputs. */
#define SW_NOALLOC_SCRATCH_BYTES (72u << 20)
int sw_advance_noalloc(const sw_grid *grid, const sw_params *params, float manning, float d50,
                       float psi, float *h, float *hu, float *hv, float *b, int32_t nsteps,
                       double dt_fixed, double t0, double *t_out, int32_t *err_out,
                       void *hip_stream, char *errbuf, int32_t errbuf_len);

/* ------------------------------------------------------------------------
 * Ensembles: many grids (uneven sizes, own terrain, soil, inflow and Eq. 7
 * step) advanced together.  Each step is one launch of the Eq. 7 reduction
 * (one workgroup per member) and one launch per stage over a table of all
 * members' tiles, replayed from a HIP graph.  Each member computes exactly
 * what it computes alone (bit for bit).
 * ------------------------------------------------------------------------ */
typedef struct swb_ctx swb_ctx;

/* Group n member solvers made by sw_create and loaded with the sw_set_*
 * calls.  Members must share one HIP stream, be distinct, and not use
 * SW_FLAG_UNFUSED.  The batch references the members and does not own them:
 * destroy the batch before its members.  Members stay usable on their own
 * (sw_get_fields, sw_get_sums, sw_set_*, sw_advance). */
int swb_create(int32_t n, sw_ctx *const *members, swb_ctx **out);
int swb_destroy(swb_ctx *batch);

/* Tile shape of every member while it is advanced by the batch (as
 * sw_set_tile_shape). */
int swb_set_tile_shape(swb_ctx *batch, int32_t tile_x, int32_t tile_y);

/* Advance every member nsteps steps, each with its own Eq. 7 step.  All
 * members must hold a state and stand at steps of the same parity
 * (SW_ERR_STATE otherwise).  Asynchronous; device errors are per member. */
int swb_advance(swb_ctx *batch, int32_t nsteps);

/* Wait for the batch; returns the first member's sticky device error. */
int swb_sync(swb_ctx *batch);

/* Batch tile-shape autotuner (the hierarchical tiling of Section 3 sized for
 * an ensemble): from the members' current states, time nsteps batch steps of
 * each tile shape, put every member's state, time and balances back, and keep
 * the fastest shape for later swb_advance calls (results are bit-identical for
 * every shape).  Members must hold states at steps of one parity
 * (SW_ERR_STATE).  Allocates and frees a copy of each member's state;
 * synchronises.  *tile_x, *tile_y (may be NULL) receive the chosen shape. */
int swb_autotune(swb_ctx *batch, int32_t nsteps, int32_t *tile_x, int32_t *tile_y);

/* Member m (0 <= m < n) of the batch, read or set through the batch: each
 * call is the member's own sw_get_fields / sw_get_sums / sw_set_* (the Main
 * block's inputs and the Save block's outputs of Section 3, per scenario),
 * with the same arguments, ordering and errors; SW_ERR_ARG for an index out of
 * range.  A new state restarts the member's step counter, so the batch then
 * advances only once all members stand at steps of one parity again. */
int swb_get_fields(swb_ctx *batch, int32_t m, float *h, float *hu, float *hv, float *b,
                   int ptr_kind);
int swb_get_sums(swb_ctx *batch, int32_t m, sw_sums *out);
int swb_set_state(swb_ctx *batch, int32_t m, const float *h, const float *hu, const float *hv,
                  int ptr_kind);
int swb_set_bed(swb_ctx *batch, int32_t m, const float *b, int ptr_kind);
int swb_set_soil(swb_ctx *batch, int32_t m, const float *manning, float manning_scalar,
                 const float *d50, float d50_scalar, const float *psi, float psi_scalar,
                 int ptr_kind);
int swb_set_inflow(swb_ctx *batch, int32_t m, const int32_t *cell_idx, const float *weight,
                   int32_t n, double q_base, double q_peak, double t_peak, double t_sigma);
int swb_set_sed_sources(swb_ctx *batch, int32_t m, const float *qb_plus, const float *qb_minus,
                        int ptr_kind);

const char *swb_last_error(const swb_ctx *batch);

#ifdef __cplusplus
}
#endif

#endif /* CSPH_H */
