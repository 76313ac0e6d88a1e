/*
 * mrs.h - C ABI of the MI355X (gfx950) library for the Method of Regularized
 * Stokeslets (MRS) on Kirchhoff-rod filaments (arxiv 2604.12083).
 *
 * The library evaluates, for every point of an ensemble of filaments, the
 * linear velocity U and angular velocity Omega induced by point forces f and
 * torques n at all points (Sec. II.C, Eqs. velocity_field,
 * angular_velocity_field, superposition), the discrete rod forces and torques
 * with the half-angle mid frame (Sec. II.B, Eqs. discrete_f, discrete_n,
 * F_comp_discrete, N_comp_discrete, mid_triad; Alg. 1; Sec. III.B.1), and
 * explicit time steps that move positions and rotate frames (Sec. III.B.3,
 * Eqs. newx, newD; Sec. III.A for the Runge-Kutta fine propagator).
 *
 * Conventions shared by every call
 * --------------------------------
 * Layout.  Positions, forces, torques, U and Omega are row-major n x 3
 *   float64 arrays (point k at [3k .. 3k+2]).  Frames are n x 9 float64 with
 *   D[9k + 3i + c] = component c of director D^{i+1} at point k (orthonormal,
 *   right-handed, D^3 the tangent).  Filaments are concatenated; `offsets`
 *   is a CSR array of n_fil + 1 int32 values, offsets[0] = 0, strictly
 *   increasing, offsets[n_fil] = n.
 * Physics.  f and n are the point force and torque exerted ON THE FLUID.
 *   Every point is a target and a source; the sum includes j = i.  eps > 0
 *   is the blob radius, mu > 0 the viscosity.  The kernel functions are those
 *   of the blob phi_eps(r) = 15 eps^4 / (8 pi (r^2 + eps^2)^{7/2}).
 * Precision.  MRS_FP64 does every operation in double precision.  MRS_FP32C
 *   evaluates each pair in single precision on hi/lo-split positions and
 *   sums with compensated single-precision accumulation per source block;
 *   the per-target sum over blocks, the rod forces, the matrix square root,
 *   the frame update and its re-orthonormalisation stay in double precision.
 * Ownership.  The caller owns every array it passes; the library copies
 *   host inputs and never keeps caller pointers past the call, except the
 *   device pointers of the *_device calls until the work queued on the
 *   given stream has finished.  The library owns the handles it returns;
 *   free them with the matching destroy call.
 * Errors.  Every call returns an mrs_status and never aborts the process.
 *   MRS_EINVAL: a null handle or pointer, n < 0, eps <= 0, mu <= 0, a
 *   non-finite scalar, a bad offsets array or an unknown enum value.
 *   MRS_ENOMEM: a device or host allocation failed.  MRS_EDEVICE: a HIP
 *   call failed (the context should then be destroyed).  MRS_ENUMERIC: a
 *   result came out non-finite (an overflow, e.g. of the single-precision
 *   source records of MRS_FP32C, or of a step): the reduction kernels raise
 *   a flag when a velocity or updated position they write is not finite,
 *   and calls that copy results to the host scan them.  It is returned by
 *   mrs_eval_host, mrs_ensemble_eval/_step/_get, mrs_batch_step/_eval,
 *   mrs_parareal(_pipelined) and by the server (result status); the
 *   results are still written.  The asynchronous *_device calls cannot
 *   report it.  mrs_last_error gives a message for the last failing call
 *   on the context.
 * Threads and streams.  A context is not thread-safe.  Calls taking a
 *   `stream` (a hipStream_t passed as void*, NULL = the context stream)
 *   are asynchronous with respect to the host; all other calls return after
 *   the device work they queued has finished unless stated otherwise.
 */
#ifndef MRS_H
#define MRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MRS_OK = 0,
    MRS_EINVAL = -1,
    MRS_ENOMEM = -2,
    MRS_EDEVICE = -3,
    MRS_ENOTREADY = -4,
    MRS_EBUSY = -5,
    MRS_ENUMERIC = -6
} mrs_status;

typedef enum { MRS_FP64 = 0, MRS_FP32C = 1 } mrs_precision;

/* Forward Euler (Eqs. newx, newD), the second-order Runge-Kutta method of
 * the paper's fine propagator (Sec. III.A, n = 2; midpoint rule) and the
 * classical four-stage Runge-Kutta method.  Runge-Kutta stage states are
 * X_s = X + c_s dt U_{s-1}, D_s = Rod(c_s dt k_{s-1}) D; a step ends with
 * X += dt sum w_s U_s, D = Rod(dt sum w_s k_s) D (Rod = Eq. newD), where
 * k_s = Omega_s for RK2 and, for RK4, the Runge-Kutta-Munthe-Kaas form
 * k_0 = Omega_0, k_s = Omega_s - theta_s x Omega_s / 2 +
 * theta_s x (theta_s x Omega_s) / 12 with theta_s = c_s dt k_{s-1}.  Orders:
 * 1, 2 and 4 in positions and frames, also with the rod forces on (without
 * the correction the RK4 frames, and through the rod forces the positions,
 * would be second order once Omega varies within a step). */
typedef enum { MRS_EULER = 1, MRS_RK2 = 2, MRS_RK4 = 4 } mrs_integrator;

/* Rod moduli (Sec. II.A, Eq. constitutive_N_F): a = bending, bending, twist;
 * b = shear, shear, stretch; omega0 = intrinsic strain-twist vector;
 * ds = arclength spacing of the discretisation (Sec. II.B). */
typedef struct {
    double a[3];
    double b[3];
    double omega0[3];
    double ds;
} mrs_rod_params;

typedef struct mrs_context mrs_context;
typedef struct mrs_ensemble mrs_ensemble;
typedef struct mrs_server mrs_server;

/* ---- context ---------------------------------------------------------- */

/* Create a context on HIP device `device` with its own non-blocking stream
 * (default priority).  *out receives the handle. */
mrs_status mrs_context_create(int device, mrs_context **out);
void mrs_context_destroy(mrs_context *ctx);
/* Message of the last failing call on ctx; valid until the next call. */
const char *mrs_last_error(const mrs_context *ctx);
/* Make `stream` (a hipStream_t, NULL = the context's own) the stream every
 * later call on ctx queues its work on. */
mrs_status mrs_context_set_stream(mrs_context *ctx, void *stream);
/* Wait until all work queued on the context stream has finished. */
mrs_status mrs_context_synchronize(mrs_context *ctx);

/* ---- one-shot MRS evaluation (Eqs. velocity_field, angular_velocity_field,
 *      superposition; Alg. 2 is the paper's GPU form of it) -------------- */

/* U, Omega at all n points from f, torque at the same points.  Host arrays
 * (n x 3), synchronous.  n = 0 is allowed and does nothing. */
mrs_status mrs_eval_host(mrs_context *ctx, int64_t n, const double *X, const double *f,
                         const double *torque, double eps, double mu, mrs_precision prec,
                         double *U, double *Omega);

/* Same on caller-owned device arrays (n x 3 each), queued on `stream`.
 * The evaluation scratch (source records, split-K partial sums, work list)
 * belongs to the context: each call makes its stream wait for the end of
 * the previous call's kernels (an event), so calls queued on different
 * streams without a host synchronisation between them run one after the
 * other on the device and each gives its own result.  The outputs are not
 * checked for finiteness (the call returns before they exist). */
mrs_status mrs_eval_device(mrs_context *ctx, int64_t n, const double *dX, const double *df,
                           const double *dtorque, double eps, double mu, mrs_precision prec,
                           double *dU, double *dOmega, void *stream);

/* mrs_eval_device for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, layouts, ordering and results, but the source records,
 * split-K partial sums and work list live in a static device array of
 * 64 MiB that the library holds on every device it runs on until the
 * process ends (its address is taken when a context is created on the
 * device); the call allocates no device or pinned host memory.  It serves at
 * most 500,000 points (MRS_EINVAL beyond, with a message); when the default
 * decomposition's partial sums do not fit, it uses fewer, longer source
 * chunks (same results up to the rounding of the split-K sum).  Nothing in
 * the array needs to start at zero; it keeps the last call's contents.  All
 * calls on one device share the array: calls of one context are ordered by
 * its evaluation event whatever their streams, but calls of different
 * contexts that overlap on the device race and give wrong results. */
mrs_status mrs_eval_device_noalloc(mrs_context *ctx, int64_t n, const double *dX, const double *df,
                                   const double *dtorque, double eps, double mu, mrs_precision prec,
                                   double *dU, double *dOmega, void *stream);

/* ---- rod mechanics (Sec. II.B, Alg. 1, Sec. III.B.1) ------------------- */

/* Point force g and torque m exerted on the fluid by every node:
 * g_k = F_{k+1/2} - F_{k-1/2} + fext_k,
 * m_k = N_{k+1/2} - N_{k-1/2} + (dX_{k+1/2} x F_{k+1/2} + dX_{k-1/2} x F_{k-1/2})/2 + next_k,
 * i.e. -ds times the paper's fluid-on-rod densities f_k, n_k, with F, N of
 * the absent end segments zero (free ends).  `offsets` is a host array;
 * dX (n x 3), dD (n x 9), dfext, dnext (n x 3, may be NULL = zero), dg, dm
 * (n x 3) are device arrays.  Queued on `stream`. */
mrs_status mrs_rod_forces_device(mrs_context *ctx, int32_t n_fil, const int32_t *offsets,
                                 const double *dX, const double *dD, const mrs_rod_params *rod,
                                 const double *dfext, const double *dnext, double *dg, double *dm,
                                 void *stream);

/* Principal square roots S (rotation by half the angle about the same axis,
 * Eq. halfangle) of `count` proper rotations R.  dR, dS: device arrays of
 * count row-major 3x3 float64 matrices.  At an angle of exactly pi either
 * root may be returned.  Queued on `stream`. */
mrs_status mrs_rotsqrt_device(mrs_context *ctx, int64_t count, const double *dR, double *dS,
                              void *stream);

/* ---- device-resident ensembles ---------------------------------------- */

/* Copy a filament ensemble to the device: offsets (n_fil + 1), X (n x 3),
 * D (n x 9), external point loads f_ext, n_ext (n x 3, NULL = zero; held
 * constant during steps), eps, mu and the rod moduli.  The device copy keeps
 * the filaments in a spatial order of the library's choosing (by the Morton
 * key of their centroids at creation, filaments whole), so that the pair
 * kernels' blocks of consecutive points stay compact; every array passed to
 * or returned by the ensemble calls uses the caller's order, and the order
 * in which the caller lists the filaments does not change any result. */
mrs_status mrs_ensemble_create(mrs_context *ctx, int32_t n_fil, const int32_t *offsets,
                               const double *X, const double *D, const double *f_ext,
                               const double *n_ext, double eps, double mu,
                               const mrs_rod_params *rod, mrs_ensemble **out);
/* Replace the state (host arrays; either may be NULL to keep it). */
mrs_status mrs_ensemble_set_state(mrs_ensemble *ens, const double *X, const double *D);
/* Replace the external point force f_ext and torque n_ext exerted on the
 * fluid at every point (Sec. II.C, Eq. superposition: the loads the MRS sum
 * takes besides the rod's own forces), n x 3 host arrays in the caller's
 * order, copied; NULL = zero.  They stay constant during later steps and
 * are added to the elastic loads (or used alone with include_elastic = 0).
 * Errors: MRS_EINVAL for a null ensemble or a non-finite value;
 * MRS_ENOMEM if an ensemble created without loads cannot get their
 * buffers. */
mrs_status mrs_ensemble_set_external(mrs_ensemble *ens, const double *f_ext, const double *n_ext);
/* Number of points. */
mrs_status mrs_ensemble_size(const mrs_ensemble *ens, int64_t *n);
/* Swimming (Sec. IV).  wave = (A, k, f), or NULL to switch it off: the
 * preferred strain-twist of segment k+1/2 becomes omega0 +
 * (0, -k^2 A sin(k s + f t), 0) at its midpoint arclength s = (k + 1/2) ds
 * and at the time t of the stage (step start + c_s dt for RK stage s).
 * lj = (sigma, energy), or NULL to switch it off: points of different
 * filaments closer than r_c = 2^(1/6) sigma repel with the force
 * -grad of 4 energy ((sigma/r)^12 - (sigma/r)^6), added to the point force
 * the node exerts on the fluid (with or without the elastic forces).
 * Host arrays, copied.  Errors: MRS_EINVAL for non-finite values,
 * sigma <= 0 or energy < 0; MRS_ENOMEM for the LJ buffers (3 doubles,
 * one int32 per point).  Cached plans and graphs of the ensemble are rebuilt
 * at its next launch. */
mrs_status mrs_ensemble_set_swimming(mrs_ensemble *ens, const double *wave, const double *lj);
/* The ensemble clock: the time of the start of its next step (0 at
 * creation).  Every step advances it by dt on the device, so that graph
 * replays and batched steps keep it; MRS_EINVAL for a non-finite t. */
mrs_status mrs_ensemble_set_time(mrs_ensemble *ens, double t);
mrs_status mrs_ensemble_get_time(mrs_ensemble *ens, double *t);
/* U, Omega at the current state from the rod forces (if include_elastic)
 * plus the external loads. */
mrs_status mrs_ensemble_eval(mrs_ensemble *ens, mrs_precision prec, int include_elastic);
/* nsteps explicit steps of size dt.  Every step ends with the frame
 * re-orthonormalisation D3 <- D3/|D3|, D1 <- unit(D1 - (D1.D3) D3),
 * D2 <- D3 x D1.  After the call U, Omega hold the first-stage velocities
 * of the last step. */
mrs_status mrs_ensemble_step(mrs_ensemble *ens, mrs_integrator integ, double dt, int32_t nsteps,
                             mrs_precision prec, int include_elastic);
/* Copy state and last velocities to host arrays (any may be NULL). */
mrs_status mrs_ensemble_get(mrs_ensemble *ens, double *X, double *D, double *U, double *Omega);
void mrs_ensemble_destroy(mrs_ensemble *ens);

/* ---- batching --------------------------------------------------------- */

/* Advance n_ens independent ensembles (e.g. the fine-propagator time slices
 * of one Parareal iteration, Sec. II.D) together: every kernel of a stage
 * covers all of them, and with use_graph != 0 the nsteps x stages launch
 * sequence is captured once into a HIP graph and replayed.  Ensembles never
 * interact; each result equals the one of mrs_ensemble_step on it alone.
 * All ensembles must belong to ctx and be distinct. */
mrs_status mrs_batch_step(mrs_context *ctx, int32_t n_ens, mrs_ensemble *const *ens,
                          mrs_integrator integ, double dt, int32_t nsteps, mrs_precision prec,
                          int include_elastic, int use_graph);
/* One U, Omega evaluation of every listed ensemble in one launch sequence. */
mrs_status mrs_batch_eval(mrs_context *ctx, int32_t n_ens, mrs_ensemble *const *ens,
                          mrs_precision prec, int include_elastic);

/* ---- serving (continuous batching) ------------------------------------ */

/* One request: an independent filament ensemble and what to do with it.
 * kind MRS_REQ_EVAL: one U, Omega evaluation; MRS_REQ_STEPS: nsteps steps of
 * size dt with integrator `integ`.  Host arrays as in mrs_ensemble_create;
 * they are copied by mrs_server_submit. */
typedef enum { MRS_REQ_EVAL = 0, MRS_REQ_STEPS = 1 } mrs_request_kind;

typedef struct {
    int32_t kind;
    int32_t n_fil;
    const int32_t *offsets;
    const double *X, *D, *f_ext, *n_ext;
    double eps, mu, dt;
    int32_t nsteps;
    int32_t integ;
    int32_t include_elastic;
    mrs_rod_params rod;
} mrs_request;

/* Completion record.  Times are seconds on the steady (monotonic) clock:
 * submission, admission to the device, and completion of the last step. */
typedef struct {
    int32_t status;
    int32_t kind;
    int64_t n;
    int32_t steps_done;
    double t_submit, t_admit, t_done;
} mrs_result_info;

typedef struct {
    int64_t submitted, admitted, completed, rejected;
    int64_t ticks, failed_ticks;
    int64_t pairs;        /* pair interactions evaluated */
    double busy_s;        /* device time of the ticks (events around each) */
    int32_t active, queued;
    int64_t hbm_in_use, hbm_budget;
    double wall_s;        /* seconds since mrs_server_start */
} mrs_server_stats;

/* Start a server thread that owns ctx until mrs_server_stop.  It admits
 * queued requests (arrival order by default, first fit; see
 * mrs_server_set_admission) while a slot is free and their
 * device footprint fits in hbm_budget_bytes, copying their state to the
 * device on a second stream while earlier work runs; every tick is ONE
 * batched sequence that advances the admitted requests by one evaluation or
 * one step, and up to two ticks are queued on the device ahead of the host;
 * a finished request's results are copied back after its last tick without
 * stopping the device.  Device memory comes from a cache of the server
 * (hipMalloc only while it warms up, released at mrs_server_stop).  All
 * requests of a server use `prec`.
 * Each request's result equals the one it gets alone (its work is split
 * the same way in every batch).  A request larger than the whole budget
 * completes with status MRS_ENOMEM without running.  If the environment variable
 * MRS_DEBUG_FAIL_TICK=k is set, tick k is treated as failed before launch
 * and its requests are retried from their step-boundary state. */
mrs_status mrs_server_start(mrs_context *ctx, mrs_precision prec, int64_t hbm_budget_bytes,
                            int32_t max_slots, mrs_server **out);
/* Bound the work of one tick to about max_pairs pair interactions (0 = no
 * bound: every admitted request advances every tick).  With a bound, each
 * admitted request earns an equal share of the budget per tick and runs in
 * the ticks where its earned share covers one unit of its work (deficit
 * round robin): small requests advance every tick, larger ones every few
 * ticks, so a large request does not hold every small one to its pace. */
mrs_status mrs_server_set_tick_pairs(mrs_server *srv, int64_t max_pairs);
/* Order in which queued requests are admitted (first fit in that order, as
 * slots and the HBM budget allow).  MRS_ADMIT_ARRIVAL (the default):
 * arrival order.  MRS_ADMIT_LEAST_WORK: least total work (pair interactions
 * of all the request's evaluations) first, which cuts the wait of small
 * requests queued behind large ones; requests that have waited longer than
 * max_wait_s (> 0; 0 = no bound) go first, in arrival order, so no request
 * waits for ever.  Applies from the next admission on; results do not
 * depend on it.  Errors: MRS_EINVAL for another order or max_wait_s < 0. */
typedef enum { MRS_ADMIT_ARRIVAL = 0, MRS_ADMIT_LEAST_WORK = 1 } mrs_admission;
mrs_status mrs_server_set_admission(mrs_server *srv, int32_t order, double max_wait_s);
/* Any host thread.  *ticket identifies the request. */
mrs_status mrs_server_submit(mrs_server *srv, const mrs_request *req, uint64_t *ticket);
/* Non-blocking.  MRS_ENOTREADY until the request is done; then fills info,
 * copies X, D (state after the last step), U, Omega (last first-stage
 * velocities) to the caller's n x 3 / n x 9 arrays (any may be NULL) and
 * forgets the request. */
mrs_status mrs_server_poll(mrs_server *srv, uint64_t ticket, mrs_result_info *info, double *X,
                           double *D, double *U, double *Omega);
/* Like poll, but waits up to timeout_s seconds. */
mrs_status mrs_server_wait(mrs_server *srv, uint64_t ticket, double timeout_s,
                           mrs_result_info *info, double *X, double *D, double *U, double *Omega);
mrs_status mrs_server_stats_get(mrs_server *srv, mrs_server_stats *out);
/* Finish admitted work, drop queued requests, join the thread, free srv. */
mrs_status mrs_server_stop(mrs_server *srv);

/* ---- pair-kernel tuning ------------------------------------------------ */

/* How the pair kernel covers an ensemble of a given size: mode 0 = LDS-tiled
 * (targets_per_lane 1 or 2, `chunks` source chunks of equal size, 0 =
 * automatic), mode 1 = wave-split for small ensembles.  Without a stored
 * configuration the library picks one from n and the compute-unit count:
 * wave-split up to 1,024 points, else one target per lane (FP32C, and
 * FP64 when two would give fewer than three blocks per
 * compute unit) or two, and source chunks of 128 sources or more (64 when
 * 128 would give at most one block per compute unit).  An automatic FP32C
 * configuration of a large grid
 * also splits the last ~8% of every target tile's sources into shorter
 * chunks dispatched last, and a tiled configuration of at least 48 blocks
 * per compute unit (24 for FP64 at two targets per lane) runs the
 * persistent schedule; mrs_tune_get reports
 * `chunks` as the total number of chunks (partial sums per target). */
typedef struct {
    int32_t mode;
    int32_t targets_per_lane;
    int32_t chunks;
    int32_t schedule;  /* tiled mode: 0 = one block per (target tile, source
                          chunk); 1 = persistent: a grid of the blocks the
                          device keeps resident, each claiming the next block
                          of the work list from a counter until none is left
                          (same results: every block of work writes its own
                          partial sums) */
} mrs_pair_config;

/* Time candidate configurations on a seeded synthetic ensemble of n points
 * (straight 128-point filaments at the density of 100 in a box of side 10)
 * in precision `prec` and store the fastest for every n of the same
 * power-of-two size class.  The candidates are the automatic configuration
 * itself (stored as chunks = 0, which keeps its chunking and tail split),
 * one and two targets per lane with automatic chunking on either schedule
 * and with the chunk counts that give 1 to 64 blocks per compute unit, the
 * four-wave split (FP32C) and, up to 8,192 points, the wave-split mode.
 * The time of a candidate is the device time of one mrs_eval_device call
 * (every kernel of it).  Every candidate runs once; the fastest quarter (at
 * least four) and the automatic configuration then run `reps` (1..20)
 * more times each, interleaved, and the medians decide.  The automatic
 * configuration is kept unless another is more than 1% faster, so a tuned
 * size class is never measurably slower than an untuned one.  *best (may be
 * NULL) receives the stored configuration and *best_ms its median time.
 * Ensembles already planned keep the configuration they were planned with.
 * With a table file set by mrs_tune_on_first_use the file is rewritten. */
mrs_status mrs_autotune(mrs_context *ctx, int64_t n, mrs_precision prec, int32_t reps,
                        mrs_pair_config *best, double *best_ms);
/* Tune on first use: with reps > 0, a size class without a stored
 * configuration is tuned (mrs_autotune with `reps`) when a plan of an
 * ensemble of that class is first built, i.e. on the first
 * mrs_ensemble_eval, mrs_ensemble_step, mrs_batch_step or mrs_parareal call
 * for it in a precision, for ensembles of at most 262,144 points (a
 * tuning pass costs about 60 evaluations); reps = 0 (the default) turns
 * this off.  Never while the context's stream is being captured, and never
 * for mrs_eval_device,
 * mrs_eval_device_noalloc, mrs_eval_host or the server, which use the table
 * or the automatic configuration as it stands.  table_path (may be NULL):
 * a tuning table file (format of mrs_tune_save) that is read now if it
 * exists, written at once (with the entries now in the table) and
 * rewritten after every tuning.  Errors: MRS_EINVAL for reps outside
 * 0..20, or a table that cannot be read, cannot be written or was written
 * for another device kind (architecture name and compute-unit count). */
mrs_status mrs_tune_on_first_use(mrs_context *ctx, int32_t reps, const char *table_path);
/* Write the tuning table to `path` (text: a header line
 * "mrs-pair-tuning 1 <architecture> <compute units> <unix time>", then one
 * line per entry: precision, log2 size class, mode, targets_per_lane,
 * chunks, schedule, tuned and automatic median ms (-1 if set by hand);
 * written to a temporary file beside it and renamed over it, so that
 * readers see the old or the new table, never part of one).  Read one back with mrs_tune_load,
 * which adds its entries (replacing those of the same class) or changes
 * nothing and returns MRS_EINVAL if the file is malformed or from another
 * device kind. */
mrs_status mrs_tune_save(mrs_context *ctx, const char *path);
mrs_status mrs_tune_load(mrs_context *ctx, const char *path);
/* Host only (no device is touched): the pair-kernel work list that the
 * automatic configuration builds for one ensemble of n points on a device
 * with n_cu compute units, in dispatch order.  *mode, *targets_per_lane,
 * *chunks and *tail_start (each may be NULL) receive the configuration
 * (chunks = partial sums per target; tail_start = first source of the short
 * tail chunks, n if there are none); *n_items receives the number of
 * blocks (the schedule that runs them is reported by mrs_tune_get).  items
 * (may be
 * NULL to query the count) receives 5 int32 per block: first target,
 * targets, first source, sources, partial-sum slot.  Errors: MRS_EINVAL for
 * n < 1 or too large, n_cu < 1, an unknown precision, a null n_items, or
 * max_items below the block count (n_items is still set). */
mrs_status mrs_plan_items(int64_t n, mrs_precision prec, int32_t n_cu, int32_t *mode, int32_t *targets_per_lane,
                          int32_t *chunks, int32_t *tail_start, int32_t *items, int64_t max_items,
                          int64_t *n_items);
/* Read / set the configuration used for ensembles of n points. */
mrs_status mrs_tune_get(mrs_context *ctx, int64_t n, mrs_precision prec, mrs_pair_config *out);
mrs_status mrs_tune_set(mrs_context *ctx, int64_t n, mrs_precision prec, const mrs_pair_config *cfg);

/* ---- Parareal on one device (Sec. II.D, Eqs. initial, intermediate,
 *      serial_correct; Sec. III.A) -------------------------------------- */

/* Parareal from the current state of `ens` over n_slices time slices of
 * length fine_steps * fine_dt.  The fine propagator F takes fine_steps steps
 * of fine_integ; the coarse propagator G takes coarse_steps forward-Euler
 * steps of the same slice.  Iteration 0 is the serial coarse sweep; iteration
 * k runs F on slices k..n_slices as ONE batched launch sequence (replayed
 * from a HIP graph), then corrects slices k+1.. serially with
 * X^k_n = F(X^{k-1}_{n-1}) + G(X^k_{n-1}) - G(X^{k-1}_{n-1}) applied to the
 * positions and the frames (frames re-orthonormalised after the
 * correction).  Stops when the relative increment of the slice-boundary
 * positions (max over points of |x^k - x^{k-1}| / |x^k|) is <= tol, or after
 * max_iter iterations (max_iter <= n_slices; after n_slices iterations the
 * result equals the serial fine solution).  On return `ens` holds the state
 * at the end of the last slice; history (max_iter doubles, may be NULL)
 * receives the increments, *iters (may be NULL) the iterations done.  All
 * state stays on the device; one host copy of the positions per iteration
 * evaluates the increment.  Each propagation of slice n starts at the slice
 * boundary time (the ensemble clock plus n fine steps, accumulated as the
 * serial run would), and the clock ends at the last boundary.  The slice
 * workers (n_slices + 1 device copies of the ensemble) stay with `ens`
 * after the call, so later calls reuse them with their launch plans and
 * graphs; they are rebuilt when its loads or swimming settings change and
 * freed with it. */
mrs_status mrs_parareal(mrs_ensemble *ens, int32_t n_slices, mrs_integrator fine_integ, double fine_dt,
                        int32_t fine_steps, int32_t coarse_steps, int32_t max_iter, double tol,
                        mrs_precision prec, int include_elastic, double *history, int32_t *iters);

/* Parareal as mrs_parareal with the pipelined schedule of Sec. II.D (the
 * fine solve of a slice starts as soon as the coarse sweep has produced its
 * initial state): the slices are split into groups of `group` consecutive
 * slices (group 0: ceil(n_slices / 4)); a group's fine propagations run as
 * one batched launch sequence on one of up to three further streams of the
 * context (default priority) as soon as the sweep has produced their start
 * states, and the next sweep corrects
 * each slice as soon as its group is done, so the serial coarse sweep
 * overlaps the fine work.  The fine groups of iteration k + 1 start during
 * sweep k only once the increment of the slices swept so far exceeds tol (so
 * that no work is done that mrs_parareal would not do).  Same arguments,
 * results (bit for bit: iterates, increments, iteration count) and errors as
 * mrs_parareal, plus MRS_EINVAL for group outside [0, n_slices]. */
mrs_status mrs_parareal_pipelined(mrs_ensemble *ens, int32_t n_slices, mrs_integrator fine_integ,
                                  double fine_dt, int32_t fine_steps, int32_t coarse_steps, int32_t max_iter,
                                  double tol, mrs_precision prec, int include_elastic, int32_t group,
                                  double *history, int32_t *iters);

/* ---- kernel timing ---------------------------------------------------- */

/* When enabled, every kernel launch of the context is bracketed by HIP events
 * on the stream it is launched on.  mrs_profile_query waits for the recorded
 * events and returns the launch count and summed duration (milliseconds) of
 * the kernels whose name contains `kernel` (NULL or "" = all).  The events
 * only time: they skip the system-scope fence of a default event (no cache
 * write-back or invalidation around the timed kernel), so they make no
 * device memory visible to the host by themselves. */
mrs_status mrs_profile_enable(mrs_context *ctx, int on);
/* Restricts the bracketing to launches whose kernel name contains `kernel`
 * (NULL or "" = every launch), so that timing one kernel adds no events
 * around the others.  The string is copied.  Errors: MRS_EINVAL for a null
 * context. */
mrs_status mrs_profile_select(mrs_context *ctx, const char *kernel);
mrs_status mrs_profile_reset(mrs_context *ctx);
/* Shader clock of the device now, in MHz: one wave spins for 200,000
 * shader-clock ticks (s_memtime) and the elapsed ticks of the constant
 * 100 MHz reference clock (s_memrealtime) give the rate.  Synchronous on the
 * context stream; meant for reporting the clock beside kernel timings. */
mrs_status mrs_profile_clock(mrs_context *ctx, double *mhz);
mrs_status mrs_profile_query(mrs_context *ctx, const char *kernel, int64_t *launches,
                             double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* MRS_H */
