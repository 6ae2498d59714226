/*
 * lbfv.h -- C ABI of liblbfv: MI355X (gfx950) D2Q9 finite-volume time steps of
 * the discrete velocity Boltzmann-BGK equation, for the two schemes compared by
 * Zhu, Wang & Guo (arXiv 1511.00242):
 *
 *   DUGKS (Sec. 2.2): the tracked f~ = f - (dt/2) Omega is advanced by
 *     f~^{n+1} = f~+ - (dt/|V|) sum_faces (xi.n) f^{n+1/2} S, with the face value
 *     obtained from the half-step characteristic solution: f-bar+ traced back by
 *     h = dt/2 with a linear reconstruction, face moments, face equilibrium, and the
 *     trapezoid back-transform (Eqs. eq_update, eq_flux, eq_char, eq_trans_2).
 *   BKG (Sec. 2.3): the same update with the face value f~+(x_b - h xi), i.e. the
 *     collision step of the standard LBM followed by Lax-Wendroff streaming in
 *     finite-volume form (Eqs. bkg_collision, lwfv, bkg_fb, bkg_fv, f_left).
 *
 * Both schemes track the same variable f~, so a state may be advanced by either.
 * Boundary conditions (Sec. 2.5, Sec. 3.3): periodic, half-way bounce-back of a
 * moving no-slip wall with ghost cells by linear extrapolation, equilibrium
 * (free-stream) inflow, zero- or first-order extrapolation outflow, symmetry planes, and a
 * wall segment ending a south / north side (Sec. 3.3).
 *
 * Conventions for every function:
 *   - returns LBFV_OK (0) or a negative lbfv_status; nothing is thrown across the ABI;
 *   - pointers are host pointers unless named dev_*; input arrays are copied during
 *     the call, output arrays are caller-allocated;
 *   - host fields are FP64, row-major [ny][nx] (x fastest); distributions are SoA
 *     [9][ny][nx] in the direction order of Sec. 2.1:
 *       0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
 *     times c = sqrt(3 RT);
 *   - one context is not thread-safe; distinct contexts are independent;
 *   - stepping is asynchronous on the context's HIP stream; observables
 *     (moments, totals, residual, get_f) synchronise that stream.
 */
#ifndef LBFV_H
#define LBFV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBFV_OK = 0,
    LBFV_EINVAL = -1,        /* bad argument (NULL, size, ordering, unsupported combination) */
    LBFV_ESTATE = -2,        /* call not valid in the current state (unset side, no initial state) */
    LBFV_ENOMEM = -3,        /* device or host allocation failed */
    LBFV_EHIP = -4,          /* a HIP runtime call failed (see lbfv_last_error) */
    LBFV_EUNSTABLE = -5,     /* a non-finite value was found at a check */
    LBFV_EUNSUPPORTED = -6   /* valid request that this build does not provide */
} lbfv_status;

/* Interface-value schemes.  DUGKS and BKG are the two methods compared; CENTRAL and UPWIND
 * are the collision-free interface values of Sec. 2.4 (Eqs. cfd1, cfd2), provided to show
 * the numerical viscosity that ignoring the collision term introduces. */
enum { LBFV_DUGKS = 0, LBFV_BKG = 1, LBFV_CENTRAL = 2, LBFV_UPWIND = 3 };
enum { LBFV_WEST = 0, LBFV_EAST = 1, LBFV_SOUTH = 2, LBFV_NORTH = 3 };
enum { LBFV_X = 0, LBFV_Y = 1 };
enum { LBFV_FP64 = 0, LBFV_FP32 = 1 };
enum { LBFV_STORE_NATIVE = 0, LBFV_STORE_DEV_FP32 = 1, LBFV_STORE_DEV_BF16 = 2, LBFV_STORE_DEV_FP16 = 3 };

typedef struct lbfv_ctx lbfv_ctx;
typedef struct lbfv_batch lbfv_batch;

/* Structured mesh (Sec. 2.2 control volumes): xf[nx+1], yf[ny+1] strictly increasing
 * face coordinates, uniform or stretched.  Copied at create. */
typedef struct {
    int32_t nx, ny;
    const double *xf, *yf;
} lbfv_mesh;

/* Velocity set (Sec. 2.1): q must be 9 (D2Q9); rt = RT = c_s^2 > 0. */
typedef struct {
    int32_t q;
    double rt;
} lbfv_velset;

/* Options (NULL = defaults: FP64, native storage, rho0 = 1, check_every = 1000,
 * default stream).
 *   compute     LBFV_FP64 or LBFV_FP32 arithmetic.
 *   storage     LBFV_STORE_NATIVE stores f~ in the compute type; LBFV_STORE_DEV_* store
 *               the deviation f~_a - F_a as FP32, BF16 or FP16 (the 16-bit forms
 *               hold (f~_a - F_a)/w_a), where F_a = feq_a(rho0, U0) is the equilibrium
 *               (Sec. 2.1, Eq. equilibrium) of a reference state, U0 = 0 unless
 *               lbfv_set_reference_velocity sets it; DEV_* need FP32 compute.
 *   rho0        reference density of the deviation storage.
 *   check_every steps between the non-finite checks; 0 disables them.  A check runs
 *               at the first launch boundary at or after check_every steps since the
 *               last one (at most steps-per-launch - 1 steps later) and reads the rest
 *               direction: a non-finite value in any direction reaches it through the
 *               cell's density within one step, so the first check made at least one
 *               step after such a value appears finds it.  lbfv_totals checks all nine.
 *   hip_stream  hipStream_t to run on; NULL = the default stream. */
typedef struct {
    int32_t compute;
    int32_t storage;
    double rho0;
    int32_t check_every;
    void *hip_stream;
} lbfv_opts;

/* Create a context for one mesh.  tau: relaxation time (nu = tau RT, Eq. nu_tau);
 * dt: time step.  CFL >= 1 is allowed (stability is the caller's choice).
 * EINVAL: NULL ctx or mesh, nx or ny < 2, non-increasing faces, q != 9, rt <= 0,
 * tau <= 0, dt <= 0, 16-bit or deviation storage with FP64 compute.  Device buffers
 * are allocated on first use unless lbfv_bind_buffers supplies them. */
int lbfv_create(const lbfv_mesh *mesh, const lbfv_velset *vel, double tau, double dt,
                const lbfv_opts *opts, lbfv_ctx **ctx);
int lbfv_destroy(lbfv_ctx *ctx);

/* Eq. eq:cfl: dt = cfl * dx / (sqrt(6) c_s), dx = smallest cell size of the mesh. */
int lbfv_dt_from_cfl(const lbfv_mesh *mesh, double rt, double cfl, double *dt);

/* Boundary setters.  All four sides must be set before the first step (else ESTATE);
 * a periodic axis is set as a whole.  Changing a side is allowed between steps. */
int lbfv_set_periodic(lbfv_ctx *ctx, int axis);
/* Half-way bounce-back wall moving with (uwx, uwy) (Sec. 2.5); ghost cells by linear
 * extrapolation of f-bar+ (DUGKS) or f~+ (BKG) to the mirrored centre. */
int lbfv_set_wall(lbfv_ctx *ctx, int side, double uwx, double uwy);
/* Free stream / inflow: ghost cells hold feq(rho, u). */
int lbfv_set_inflow_eq(lbfv_ctx *ctx, int side, double rho, double ux, double uy);
/* Outflow: ghost cells copy the adjacent cell (order 0) or extrapolate linearly (order 1). */
int lbfv_set_outflow_extrap(lbfv_ctx *ctx, int side, int order);
/* Symmetry plane (Sec. 3.3: the section of the flat-plate domain's lower side ahead of the
 * plate): specular reflection.  Ghost cells hold the adjacent cell's value of the mirrored
 * direction (normal component reversed), and on the side's faces the incoming values are
 * the outgoing ones mirrored, so no mass crosses. */
int lbfv_set_symmetry(lbfv_ctx *ctx, int side);
/* No-slip wall segment at the end of a south or north side (Sec. 3.3: the plate starts at
 * its leading edge): cells first_cell..nx-1 of the side are a half-way bounce-back wall
 * moving with (uwx, uwy); the cells before it keep the side's kind, which must already be
 * set and not periodic (else EINVAL).  Setting the side's kind again removes the segment.
 * EINVAL also for an x-side, first_cell outside [0, nx) or a non-finite velocity. */
int lbfv_set_wall_from(lbfv_ctx *ctx, int side, int32_t first_cell, double uwx, double uwy);

/* State.  f~ of an equilibrium state is feq (Omega(feq) = 0). */
int lbfv_init_equilibrium(lbfv_ctx *ctx, const double *rho, const double *ux, const double *uy);
/* Chapman-Enskog initial state (Sec. 3.1): f = feq - tau (d_t feq + xi.grad feq) evaluated
 * from rho, u and their derivatives by the chain rule, stored as f~ = f - (dt/2) Omega(f).
 * drho, dux, duy: [3][ny][nx] FP64, the derivatives along (t, x, y). */
int lbfv_init_chapman_enskog(lbfv_ctx *ctx, const double *rho, const double *ux, const double *uy,
                             const double *drho, const double *dux, const double *duy);
int lbfv_set_f(lbfv_ctx *ctx, const double *f);   /* f~, [9][ny][nx] FP64 */
int lbfv_get_f(lbfv_ctx *ctx, double *f);         /* f~, [9][ny][nx] FP64 */
/* Use caller-owned device buffers (e.g. PyTorch tensors) for the two state buffers;
 * each must hold lbfv_required_bytes and outlive the context.  The current state is
 * not carried over (set it again afterwards). */
int lbfv_bind_buffers(lbfv_ctx *ctx, void *dev_a, void *dev_b, size_t bytes);
int lbfv_required_bytes(const lbfv_ctx *ctx, size_t *bytes_per_buffer);

/* Advance nsteps time steps; asynchronous on the context stream.  Returns EUNSTABLE
 * if an earlier check found a non-finite value (checks are read without waiting: a
 * call sees the result of every check the device has finished; the next check, and
 * lbfv_totals, wait for a pending one), ESTATE if a side is unset or no state has
 * been set. */
int dugks_step(lbfv_ctx *ctx, int32_t nsteps);
int bkg_step(lbfv_ctx *ctx, int32_t nsteps);
/* Any of the four schemes.  CENTRAL (Eq. cfd1): the face value is f^n interpolated to the
 * face centre; UPWIND (Eq. cfd2): f^n traced back by h along xi with the stencil of
 * Eq. f_left.  Both use f = (2 tau f~ + dt feq)/(2 tau + dt) of the cells and the same
 * update f~^{n+1} = f~+ - dt/|V| sum (xi.n) f_b S as the other two.  EINVAL for an
 * unknown scheme; otherwise as dugks_step. */
int lbfv_step(lbfv_ctx *ctx, int scheme, int32_t nsteps);

/* Observables, FP64, synchronising the stream.
 * lbfv_moments: rho = sum f~, rho u = sum xi f~ (Sec. 2.2, Eq. macro_var).
 * lbfv_totals:  out[0] = sum rho |V|, out[1..2] = sum rho u |V| (fixed reduction order).
 * lbfv_residual: ||u - u_prev||_2 / ||u||_2 over both components and all cells, where
 *               u_prev is the velocity at the previous lbfv_residual call (1.0 on the
 *               first call). */
int lbfv_moments(lbfv_ctx *ctx, double *rho, double *ux, double *uy);
int lbfv_totals(lbfv_ctx *ctx, double out[3]);
int lbfv_residual(lbfv_ctx *ctx, double *r);

/* lbfv_totals without any allocation, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Enqueues the totals reduction on the context's stream and returns without waiting.
 * dev_out: caller-owned device memory of 4 doubles; it receives sum rho |V|,
 * sum rho u |V|, sum rho v |V| (the same kernels and summation order as lbfv_totals,
 * hence the same bits) and the number of cells holding a non-finite value (the
 * context's unstable flag is not updated: the caller reads dev_out[3]).  The per-block
 * partial sums go to a fixed scratch array of the library, 1024 x 6 doubles (48 KiB),
 * one per GPU, held until the process ends; that need does not depend on the mesh size.
 * Calls that overlap on one GPU (any contexts, any streams) race on the array, so they
 * must be ordered (one stream, or events).  ESTATE before the context's mesh metrics
 * are on the device (the first step or lbfv_totals call uploads them, and that upload
 * allocates) or before a state exists; EINVAL for a NULL pointer or when the current
 * device is not the one the context was created on. */
int lbfv_totals_device(lbfv_ctx *ctx, double *dev_out);

/* Execution shape of the step kernel: rows of the row block one wavefront marches
 * through, and wavefronts per workgroup (1, 2 or 4).  0 keeps the current value. */
int lbfv_set_tile(lbfv_ctx *ctx, int32_t rows, int32_t waves_per_block);
int lbfv_get_tile(const lbfv_ctx *ctx, int32_t *rows, int32_t *waves_per_block);
/* Work split of two steps per launch: 0 (default) one wavefront per work item (strip x
 * row block) advances both steps; 1 a workgroup of two wavefronts per item, the first
 * advancing the first step (with its ghost cells) and handing each new row to the second
 * through LDS, which advances the second step and stores it.  Each then holds one step's
 * rows in registers (about half), so more wavefronts fit per SIMD and each wave's chain
 * of dependent work is half as long.  The same bits either way; waves_per_block of
 * lbfv_set_tile does not apply to the pair form.  Ignored with one step per launch.
 * EINVAL unless 0 or 1. */
int lbfv_set_wave_pairs(lbfv_ctx *ctx, int32_t on);
int lbfv_get_wave_pairs(const lbfv_ctx *ctx, int32_t *on);
/* Time steps per launch of the single-case step: 1 to 4.  With 2, each wavefront reads its
 * strip of the state once, keeps the intermediate step in registers (ghost cells, wall and
 * symmetry faces of both steps included) and writes the second, so a step moves half the
 * HBM bytes; the result is the same, bit for bit, as two one-step launches (with 16-bit
 * storage the intermediate step is not rounded to 16 bits, so the two differ).  With 3 or
 * 4 (doubly periodic meshes of at least 2 x steps cells per side) each work item is a
 * chain of that many wavefronts, one per step, handing rows on through LDS: a step moves a
 * third or a quarter of the bytes, with the same bits as one-step launches.  The state
 * moves to a strip layout of 64 - 2 x steps columns (the buffers of lbfv_required_bytes
 * hold every layout).  Steps left over at the end of a call make one launch of fewer
 * steps; if a side stops being periodic, the next step call moves to 2.  EINVAL for another
 * value, for 2 to 4 before all four sides are set, or for 3 or 4 on a mesh with a
 * non-periodic side or too few cells. */
int lbfv_set_time_block(lbfv_ctx *ctx, int32_t steps);
int lbfv_get_time_block(const lbfv_ctx *ctx, int32_t *steps);
/* Reference velocity U0 (physical units) of the deviation storage: the state is stored as
 * f~_a - feq_a(rho0, U0), so a flow near a uniform stream U0 (a free stream past a plate)
 * keeps small stored values and small FP32 rounding.  The results are those of U0 = 0 up
 * to that rounding (the step is affine and feq(rho0, U0) is a fixed point of the
 * collision); the wall bounce-back of Sec. 2.5 takes its momentum term relative to U0.
 * An existing state is re-encoded in place (rounded once).  EINVAL: non-finite values, or
 * FP64 compute (native storage, where nothing is gained).  Stepping returns ESTATE while
 * U0 has a component normal to a symmetry side (feq(rho0, U0) must be mirror-symmetric
 * there).  Batches always use U0 = 0. */
int lbfv_set_reference_velocity(lbfv_ctx *ctx, double ux, double uy);
int lbfv_get_reference_velocity(const lbfv_ctx *ctx, double *ux, double *uy);
/* Autotuner: times the candidate shapes for `scheme` on this context (the state is
 * saved and restored), keeps the fastest, and records it in a cache file keyed by
 * (gfx arch, scheme, precision, storage, time block, mesh size class).  cache_path NULL: the
 * environment variable LBFV_TUNE_CACHE, else no file.  A cached entry is used
 * without timing.  best_ms (nullable) receives the time per step of the choice. */
int lbfv_autotune(lbfv_ctx *ctx, int scheme, int32_t trial_steps, const char *cache_path,
                  double *best_ms);

const char *lbfv_strerror(int status);
const char *lbfv_last_error(const lbfv_ctx *ctx);   /* ctx NULL: last error of this thread */
const char *lbfv_batch_last_error(const lbfv_batch *b);   /* b NULL: last error of this thread */

/* ------------------------------------------------------------------------------
 * Batched form: many independent cases of uneven size, Reynolds number and boundary
 * type advanced together.  One kernel launch per time step (or per two, see
 * lbfv_batch_set_time_block) covers a flat list of (case, strip, row block) items;
 * lbfv_batch_step replays a HIP graph of K such launches.  Compute / storage follow opts (FP32 deviation storage is the
 * intended use).  bc_kind per side: 0 periodic, 1 wall (bc_val = uwx, uwy),
 * 2 inflow (rho, ux, uy), 3 outflow (order), 4 symmetry. */
typedef struct {
    lbfv_mesh mesh;
    double tau, dt;
    int32_t bc_kind[4];
    double bc_val[4][3];
} lbfv_case;

int lbfv_batch_create(int32_t n, const lbfv_case *cases, const lbfv_velset *vel,
                      const lbfv_opts *opts, lbfv_batch **batch);
int lbfv_batch_init_equilibrium(lbfv_batch *b, int32_t case_id, const double *rho,
                                const double *ux, const double *uy);
int lbfv_batch_set_f(lbfv_batch *b, int32_t case_id, const double *f);
int lbfv_batch_get_f(lbfv_batch *b, int32_t case_id, double *f);
/* Advance every case by nsteps (scheme LBFV_DUGKS or LBFV_BKG); whole multiples of
 * the graph length K run as graph replays, the rest as single launches. */
int lbfv_batch_step(lbfv_batch *b, int scheme, int32_t nsteps);
int lbfv_batch_moments(lbfv_batch *b, int32_t case_id, double *rho, double *ux, double *uy);
/* Per-case count of cells whose stored values or FP64 moments are not finite (count[n],
 * caller-allocated); synchronises the stream.  This is the per-case form of the
 * non-finite check, used to map the stable range of (CFL, dt/tau) (Sec. 3.2). */
int lbfv_batch_nonfinite(lbfv_batch *b, int32_t *count);
/* Graph length K (default 100) and rows per row block of the work list (default 8); 0
 * keeps the current value. */
int lbfv_batch_set_shape(lbfv_batch *b, int32_t graph_steps, int32_t rows);
int lbfv_batch_get_shape(const lbfv_batch *b, int32_t *graph_steps, int32_t *rows);
/* Grid form of the batch's launches: 0 (default) launches the waves that fit on the device
 * at once, which walk the work list with a stride; 1 launches one wave per work item, so
 * that the hardware gives each freed slot the next block.  Results are the same either way.
 * EINVAL for another value. */
int lbfv_batch_set_grid_form(lbfv_batch *b, int32_t wave_per_item);
int lbfv_batch_get_grid_form(const lbfv_batch *b, int32_t *wave_per_item);
/* Work split of two steps per launch in the batch, as lbfv_set_wave_pairs for one case:
 * 1 gives each work item a workgroup of two wavefronts, one per step level; the grid form
 * then counts pairs instead of waves.  The same bits either way; ignored with one step per
 * launch.  EINVAL unless 0 or 1. */
int lbfv_batch_set_wave_pairs(lbfv_batch *b, int32_t on);
int lbfv_batch_get_wave_pairs(const lbfv_batch *b, int32_t *on);
/* Time steps per launch of the batch: 1 (default) or 2, as lbfv_set_time_block for one
 * case: with 2 every case moves to the 60-column strip layout, each launch advances every
 * case by two steps with the intermediate step in registers, a graph of K launches by 2K
 * steps, and an odd step count ends with a one-step launch; the result is the same, bit
 * for bit, as with 1 (16-bit storage: as for lbfv_set_time_block).  Synchronises the
 * stream.  EINVAL for another value. */
int lbfv_batch_set_time_block(lbfv_batch *b, int32_t steps);
int lbfv_batch_get_time_block(const lbfv_batch *b, int32_t *steps);
/* Autotuner of the batch: times the time blocks 1 and 2, row-block heights of the work
 * list (2, 4, ..., 64 and the three a cost model of whole rounds of resident waves ranks
 * best) and two grid forms (the resident waves walking the list, or one wave per item) for
 * `scheme`, each as a replay of a graph of trial_steps launches after one warm-up replay;
 * keeps the fastest, and restores every case's state and the step parity (the trial steps
 * leave no trace).  Needs a device copy of the whole state for its
 * duration (ENOMEM otherwise).  best_ms (nullable) receives the time per step of the
 * choice.  EINVAL for an unknown scheme or trial_steps < 1. */
int lbfv_batch_autotune(lbfv_batch *b, int scheme, int32_t trial_steps, double *best_ms);
int lbfv_batch_info(const lbfv_batch *b, int64_t *total_cells, int32_t *work_items);
int lbfv_batch_destroy(lbfv_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBFV_H */
