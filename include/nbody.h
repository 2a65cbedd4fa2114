/*
 * nbody.h -- C ABI of libnbody, the MI355X (gfx950) direct-summation N-body force and
 * Hermite block-step library.
 *
 * The method is the one of Portegies Zwart, Belleman & Geldof (2007), "High Performance Direct
 * Gravitational N-body Simulations on Graphics Processing Units": a fourth-order Hermite
 * predictor-corrector with power-of-two block time steps (Sec. 2), whose cost is the direct
 * sum of acceleration, jerk and potential on the active block (Sec. 2 Eq. Force, with the
 * softening of App. A).
 *
 * Conventions shared by every call
 *   - All array pointers are DEVICE pointers on the current HIP device unless a parameter says
 *     "host".  The caller owns every pointer it passes; the library never frees them and keeps
 *     them only between nb_bind() (or nb_bind_scratch()) and the next such call or
 *     nb_destroy().
 *   - The library allocates no device memory.  Besides the particle state, a context works in
 *     one caller-owned workspace of nb_scratch_bytes() bytes (j-particle stream, block list,
 *     scheduler record, j-split partial sums, energy and adjoint scratch), bound with
 *     nb_bind_scratch(); an ensemble likewise (nb_ens_scratch_bytes(), nb_ens_bind_scratch()).
 *     The library owns only its host-side context, captured HIP graphs and one private
 *     capture stream per context (an ensemble split into lanes also the lanes' streams and
 *     events and a pinned host copy of its cluster records per lane).
 *   - Per-particle vectors are structure-of-arrays: component c (0 = x, 1 = y, 2 = z) of
 *     particle i lives at [c * ld + i], where ld is the array's leading dimension (n for the
 *     particle state, the caller's n_i_max for force outputs).
 *   - Time is an int64 count of ticks of 2^-lmax (the smallest time step); a particle on level
 *     l has time step 2^-l = 2^(lmax - l) ticks; lmin <= l <= lmax.
 *   - Every call is asynchronous on the stream set by nb_set_stream() (default: the null
 *     stream), except nb_energy(), nb_sync() and nb_read_control(), which synchronise it.
 *   - Errors: each call returns an nb_status.  Argument errors are detected before anything is
 *     enqueued.  Conditions the device detects (a non-finite force, a step that wanted to be
 *     below 2^-lmax) are latched in a device flag word and reported by the next synchronising
 *     call.  nb_last_error() gives a message for the last failing call on a context.
 *   - A context is not thread-safe; use one context per host thread.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nb_ctx nb_ctx;

typedef enum {
    NB_OK = 0,
    NB_EINVAL = -1,     /* bad argument (NULL pointer, size out of range, unbound state)   */
    NB_EDEVICE = -2,    /* a HIP runtime call failed; nb_last_error() has its message      */
    NB_ENOMEM = -3,     /* device allocation failed                                        */
    NB_ESTATE = -4,     /* call out of order (e.g. nb_correct before any nb_force)          */
    NB_ENONFINITE = -5, /* a force or corrected state was not finite (device flag)         */
    NB_EDTMIN = -6      /* the time-step criterion asked for less than 2^-lmax (clamped)   */
} nb_status;

/* Arithmetic of the pair interaction (the rest of the step is always IEEE double).
 *  NB_FP32: single-precision VALU arithmetic; separations formed from double positions and
 *           then rounded once; sums over j-tiles accumulated in float and folded into double.
 *  NB_DS:   double-single (float-float) arithmetic throughout the interaction and its sums.
 *  NB_FP64: IEEE double arithmetic throughout.
 *  NB_FP32_ALL: the arithmetic of the paper's GPU kernel (Sec. Mapping, Appendix A):
 *           predicted positions, velocities and masses rounded to float, separations formed
 *           in float, sums over all j in float.  Single contexts only (not ensembles, not the
 *           shared-step and adjoint calls); a reference point for accuracy studies.
 *  NB_FP32_FIXED: the NB_FP32 interaction with order-independent sums: float sums over aligned
 *           64-j sub-blocks added into int64 fixed point (acc and pot 2^-44, jerk 2^-42; the
 *           idea of the GRAPE-6 accumulators the paper compares with), so forces are bitwise
 *           identical for every launch variant and j-split.  Sums beyond the fixed-point range
 *           (|acc|, |pot| >= 2^19, |jerk| >= 2^21; enough for total mass 1 and eps >= 1e-3)
 *           are reported as NB_ENONFINITE.  Single contexts only, as NB_FP32_ALL. */
typedef enum {
    NB_FP32 = 0, NB_DS = 1, NB_FP64 = 2, NB_FP32_ALL = 3, NB_FP32_FIXED = 4
} nb_precision;

/* FP64 master state of n particles, caller-owned device memory (structure of arrays). */
typedef struct {
    double *x;      /* 3*n positions                                                        */
    double *v;      /* 3*n velocities                                                       */
    double *a;      /* 3*n accelerations at each particle's own time                        */
    double *k;      /* 3*n jerks (time derivative of the acceleration)                      */
    double *m;      /* n masses                                                             */
    double *pot;    /* n potentials, from the particle's last force evaluation             */
    int64_t *tick;  /* n particle times (ticks)                                             */
    int32_t *level; /* n time-step levels                                                   */
} nb_state;

/* Device-resident scheduler record, readable with nb_read_control(). */
typedef struct {
    int64_t t_cur;        /* time of the last completed block step (ticks)                  */
    int64_t t_next;       /* time of the block currently selected (ticks)                   */
    int64_t t_end;        /* nb_run() stops selecting blocks beyond this time               */
    int64_t n_steps;      /* block steps completed since nb_init()                          */
    int64_t n_active_sum; /* sum of block sizes over those steps                            */
    int32_t n_act;        /* size of the selected block                                     */
    int32_t flags;        /* bit 0: non-finite value seen; bit 1: step clamped at 2^-lmax;
                             bit 2: block selection found a particle behind the block time   */
} nb_control;

/* Create a context for n particles (1 <= n <= 2^28) with Plummer softening eps >= 0, largest
 * step 2^-lmin and smallest step 2^-lmax (0 <= lmin <= lmax <= 52), interaction arithmetic
 * `precision`, on the current device.  Allocates no device memory (see nb_bind_scratch).
 * *out is set to NULL on failure. */
nb_status nb_create(nb_ctx **out, int32_t n, double eps, int32_t lmin, int32_t lmax,
                    int32_t precision);

/* Bytes of device workspace a context of n particles and this precision needs on the current
 * device (the j-split partial sums are sized from its compute-unit count; 256, the MI355X's,
 * when no device is visible): about 300 bytes per particle plus the partial sums (at most 64
 * j-ranges of 56 bytes per particle for full-force calls).  0 if the arguments are invalid.
 * Needs no device and allocates nothing. */
size_t nb_scratch_bytes(int32_t n, int32_t precision);

/* Bind the context's workspace: `bytes` >= nb_scratch_bytes(n, precision) of caller-owned
 * device memory at a 256-byte aligned address (e.g. a torch tensor), which the library
 * carves into its work buffers and initialises (on the context's stream).  Required before
 * any call that enqueues work; binding another workspace drops the state of the old one
 * (scheduler record, predicted stream, captured graph).  NB_EINVAL if too small or misaligned. */
nb_status nb_bind_scratch(nb_ctx *ctx, void *scratch, size_t bytes);

/* Release the context (never the caller's memory).  NULL is a no-op. */
nb_status nb_destroy(nb_ctx *ctx);

/* Enqueue subsequent work on `hip_stream` (a hipStream_t; NULL = the null stream). */
nb_status nb_set_stream(nb_ctx *ctx, void *hip_stream);

/* Bind the caller's FP64 state arrays (all fields required, each sized for n particles). */
nb_status nb_bind(nb_ctx *ctx, const nb_state *state);

/* Sec. 2 start of a run: full force on all n particles from x, v, m at time 0, then the
 * initial step of each particle, Eq. initTimestep: dt = eta |a| / |k|, rounded down to a power
 * of two in [2^-lmax, 2^-lmin].  Writes a, k, pot, level; sets every tick to 0.  Resets the
 * scheduler record and selects the first block. */
nb_status nb_init(nb_ctx *ctx, double eta);

/* Sec. 2 block selection with Eq. timestep.  First gives each particle of the block corrected
 * last its new level from dt = (eta (|a1||a2p| + |k1|^2) / (|k1||a3| + |a2p|^2))^(1/2): the
 * step halves until it is not above dt, or doubles once when dt allows twice the old step, the
 * particle's time is a multiple of the doubled step and the doubled step is at most 2^-lmin.
 * Then selects the next block: t_next = min_i (t_i + dt_i) and the block {i : t_i + dt_i =
 * t_next}, in ascending index order, kept on the device (see nb_active()).  A block beyond
 * the scheduler's t_end is not selected (its size is 0). */
nb_status nb_schedule_block(nb_ctx *ctx, double eta);

/* Device pointers to the selected block: index list (int32, capacity n) and its length. */
nb_status nb_active(nb_ctx *ctx, const int32_t **idx, const int32_t **n_act);

/* Sec. 2 predictor: x_p = x + v D + a D^2/2 + k D^3/6 and v_p = v + a D + k D^2/2 of all n
 * particles, D = (t - t_i) 2^-lmax, in double precision, stored as the j-particle stream the
 * force reads (precision-dependent layout, library-owned).  `t` is a device pointer to an
 * int64 tick count; NULL means the selected block time t_next. */
nb_status nb_predict(nb_ctx *ctx, const int64_t *t);

/* Sec. 2 Eq. Force with App. A softening, on the predicted stream: for each listed i,
 *   acc_i  =  sum_{j != i} m_j d s^(-3/2),
 *   jerk_i =  sum_{j != i} m_j [u s^(-3/2) - 3 (d.u) d s^(-5/2)],
 *   pot_i  = -sum_{j != i} m_j s^(-1/2),
 * with d = x_j - x_i, u = v_j - v_i, s = |d|^2 + eps^2, over all n predicted j-particles.
 * i_idx: device int32 list of particle indices (NULL: 0, 1, ..., n_i - 1).
 * n_i:   device int32 count (NULL: use n_i_max); must not exceed n_i_max.
 * acc, jerk: 3 * n_i_max doubles (leading dimension n_i_max); pot: n_i_max doubles.
 * Rows at and beyond the device count are left untouched.  Requires a prior nb_predict(). */
nb_status nb_force(nb_ctx *ctx, const int32_t *i_idx, const int32_t *n_i, int32_t n_i_max,
                   double *acc, double *jerk, double *pot);

/* For callers that cannot allocate device memory or take it from the caller's workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation): nb_force with
 * the same arguments and bitwise the same results, whose j-split partial sums go to a static
 * device array of 64 MiB per GPU (held from the first nb_create on that GPU until the process
 * ends) instead of the context's workspace.  Allocates nothing.  NB_EINVAL, before anything is
 * enqueued, if the call's j-split needs more than the array holds (7 doubles per partial row;
 * with a device count the largest count up to n_i_max is assumed): all block-step lists fit at
 * n = 65536, a full-force call on 2^20 particles (16 j-ranges) does not.  The array's contents
 * need no clearing (every partial row a call reads, the same call has written), but every call
 * on one GPU shares it: calls that overlap on one GPU (other streams, other contexts) race. */
nb_status nb_force_noalloc(nb_ctx *ctx, const int32_t *i_idx, const int32_t *n_i,
                           int32_t n_i_max, double *acc, double *jerk, double *pot);

/* Sec. 2 corrector of the selected block over its steps, in double precision: from the old
 * a0, k0 and the new acc/jerk (as written by nb_force on nb_active()'s list, leading dimension
 * n), a2 = -6 (a0 - a1)/dt^2 - (4 k0 + 2 k1)/dt, a3 = 12 (a0 - a1)/dt^3 + 6 (k0 + k1)/dt^2,
 * x = x_p + a2 dt^4/24 + a3 dt^5/120, v = v_p + a2 dt^3/6 + a3 dt^4/24, with x_p, v_p
 * recomputed in double.  Stores a1, k1, pot; sets each block particle's time to t_next; keeps
 * the time-step criterion inputs for the next nb_schedule_block(). */
nb_status nb_correct(nb_ctx *ctx, const double *acc, const double *jerk, const double *pot);

/* One whole block step, nsteps times, with bitwise the result of nb_schedule_block, nb_predict,
 * nb_force on the block (library-owned outputs) and nb_correct, in three launches: the block
 * selection fused with the predictor, the force, and its j-split reduction fused with the
 * corrector and the new levels.  The block list this builds (nb_active) holds the same
 * particles as the separate calls' but in no fixed order across chunks of the particle range;
 * no result depends on that order.  Particles on one level share their time (the
 * rules above keep t_i a multiple of dt_i), so the block time is the first multiple of the
 * finest occupied step after the current time, read from a per-level count the step keeps on
 * the device; a particle found behind it latches an error (NB_ESTATE at the next synchronising
 * call).  Afterwards the block just corrected already has its new levels.  With use_graph != 0
 * the step is captured once into a HIP graph and replayed. */
nb_status nb_step(nb_ctx *ctx, double eta, int32_t nsteps, int32_t use_graph);

/* Advance block steps until the block time would pass t_end (ticks): the scheduler selects no
 * block beyond t_end, so the run ends exactly at the last block time <= t_end.  Runs at most
 * max_steps steps (<= 0: no limit), synchronising once per `chunk` steps (chunk >= 1) to test
 * for completion.  Returns NB_OK, or a latched device error. */
nb_status nb_run(nb_ctx *ctx, double eta, int64_t t_end, int64_t max_steps, int32_t chunk,
                 int32_t use_graph);

/* nb_run's path for small contexts: with n <= max_n (default 1024; 0: never), softening
 * eps > 0 and the FP32, double-single or FP64 arithmetic, nb_run advances the particles with
 * one resident workgroup that keeps the FP64 state in LDS and repeats the whole block step (the
 * block of Sec. 2, the force of Eq. Force on it with every particle predicted as it is staged,
 * the corrector and the new levels of Eq. timestep) up to `chunk` times per launch, instead of
 * a chain of launches per step; the state is written back at the end of each launch.  The same
 * steps up to the summation order; nb_run does not write the j-particle stream then (call
 * nb_predict before a later nb_force).  NB_EINVAL for max_n outside [0, 1024] (the largest
 * state one workgroup's LDS holds). */
nb_status nb_set_resident(nb_ctx *ctx, int32_t max_n);

/* Sec. 4.2 energy diagnostic, synchronising: kinetic sum m v^2 / 2 and softened potential
 * energy -1/2 sum_i sum_{j != i} m_i m_j s^(-1/2), in double precision, of the state predicted
 * to the last completed block time (exact at times where all particles are synchronised).
 * ekin, epot are HOST pointers. */
nb_status nb_energy(nb_ctx *ctx, double *ekin, double *epot);

/* Copy the device scheduler record to the HOST struct *out (synchronising), and return the
 * latched device error, if any: NB_ENONFINITE, NB_ESTATE from the block selection or
 * NB_EDTMIN, with *out filled in those cases too (its flags say which).  NB_ESTATE without a
 * bound workspace leaves *out untouched. */
nb_status nb_read_control(nb_ctx *ctx, nb_control *out);

/* Force-kernel timing for measurement: with enable != 0, every force-kernel launch of this
 * context is bracketed by HIP events recorded on the context's stream (nb_step then launches
 * eagerly instead of through a graph).  Enabling or disabling discards earlier records;
 * synchronising. */
nb_status nb_profile(nb_ctx *ctx, int32_t enable);

/* Total milliseconds between the bracketing events and the number of timed force launches
 * since profiling was enabled (HOST outputs), for full-force launches (which = 0, the nb_init
 * force and nb_force calls without a device count on more than n/8 particles), the other
 * launches (which = 1: block steps and small lists) or all (which = -1).  The two classes are
 * also distinct kernel symbols.  Synchronising. */
nb_status nb_profile_read(nb_ctx *ctx, int32_t which, double *ms_total, int64_t *launches);

/* ------------------------------------------------------------------------------------------
 * Shared-step runs and their derivatives (fp32 and fp64 contexts).
 * A shared step advances every particle by the same dt = 2^-l (lmin <= l <= lmax): the
 * predictor, the force on all particles and the corrector of Sec. 2 with that dt.  Start a run
 * with nb_init (it sets a, k from the force at time 0).
 * ------------------------------------------------------------------------------------------ */
nb_status nb_shared_step(nb_ctx *ctx, double dt, int32_t nsteps);

/* Vector-Jacobian product of the force on all particles (Sec. 2 Eq. Force with App. A
 * softening) at the predicted stream (call nb_predict first): given abar, kbar (3n each,
 * adjoints of the accelerations and jerks), ADDS to xbar, vbar (3n, adjoints of the predicted
 * positions and velocities) and mbar (n, adjoints of the masses) the derivative of
 * sum_i abar_i . acc_i + kbar_i . jerk_i.  Structure of arrays, leading dimension n. */
nb_status nb_force_vjp(nb_ctx *ctx, const double *abar, const double *kbar, double *xbar,
                       double *vbar, double *mbar);

/* Vector-Jacobian product of one shared step of size dt taken from the bound state (x, v, a,
 * k: the state BEFORE the step; it is not modified).  On entry xbar, vbar, abar, kbar (3n
 * each) hold the adjoints of the step's outputs (x', v', a', k'); on return, the adjoints of
 * its inputs (x, v, a, k).  mbar (n) accumulates the masses' adjoint.  Uses the context's own
 * scratch and the j-particle stream. */
nb_status nb_step_vjp(nb_ctx *ctx, double dt, double *xbar, double *vbar, double *abar,
                      double *kbar, double *mbar);

/* Force-kernel launch variant: i-particles held per work-item (ipl), unroll of the j-loop,
 * desired number of equal work items per launch (target; the j-range is split K ways when the
 * i-blocks alone are fewer), the largest split (kmax), and the fewest j-tiles of 256 in a work
 * item whose j-records the float modes read with wave-uniform scalar loads (scalar_tiles, at
 * least 1; shorter items stage the j-records in LDS; FP64 always stages them; in
 * nb_set_variant, 0 keeps the current value).  Compiled: fp32 ipl in {1, 2} with unroll in
 * {1, 2, 4}, and ipl = 4 with unroll in {1, 2}; fixed-point ipl in {1, 2} with unroll in {1, 2};
 * ds, fp64 and all-single ipl = 1 and unroll in {1, 2}.  Any choice computes the same sums up to
 * rounding order (fixed-point: bitwise the same); scalar_tiles never changes a result. */
typedef struct {
    int32_t ipl, unroll, target, kmax, scalar_tiles;
} nb_variant;

/* The variant used for force calls on (nearly) all particles (which = 0: nb_init, nb_force
 * without a device count on more than n/8 particles) or for block-step and other calls
 * (which = 1). */
nb_status nb_get_variant(nb_ctx *ctx, int32_t which, nb_variant *out);

/* Replace that variant (HOST struct).  NB_EINVAL if it is not compiled, if its target exceeds
 * 256 work items per compute unit, or if its j-split would need more partial-sum storage than
 * the context holds (sized for one or two i per work-item with up to 16 items per compute unit
 * and any split, up to 256 items per compute unit and at most 64 j-ranges with one i per
 * work-item, or up to 128 with two). */
nb_status nb_set_variant(nb_ctx *ctx, int32_t which, const nb_variant *v);

/* Autotuner: launch every available variant (scalar_tiles 1, 4 or 16 in the float modes) on
 * the first n_i particles against the predicted stream (which = 0: count passed from the host;
 * which = 1: count read from device memory, as block steps do), `reps` timed launches each after one untimed, keep the fastest
 * for `which`, and return it in *best with its mean time in milliseconds (HOST outputs, either
 * may be NULL).  Overwrites the library's own force outputs only.  Synchronising; requires a
 * prior nb_predict(). */
nb_status nb_tune(nb_ctx *ctx, int32_t which, int32_t n_i, int32_t reps, nb_variant *best,
                  double *best_ms);

/* Calibration for measurement (not part of the method): the FP32 fused multiply-add rate of
 * the device in TFLOP/s (HOST output), from a kernel of 16 independent two-operand FMA chains
 * per work-item over 64 workgroups of 256 per compute unit, the multiplier a scalar or a vector
 * operand, best of ten timed launches (after two untimed) on the context's stream.  Requires a
 * bound workspace; synchronising. */
nb_status nb_fma_rate(nb_ctx *ctx, double *tflops);

/* Wait for the context's stream; returns a latched device error, if any. */
nb_status nb_sync(nb_ctx *ctx);

/* ------------------------------------------------------------------------------------------
 * Ensembles: many independent clusters, each integrated by its own Sec. 2 block-step scheme
 * (own particle times, levels and blocks), advanced together.  One global step gives every
 * cluster that has not reached t_end one of its own block steps: the force work items of all
 * clusters' blocks spread over the whole GPU (j- and i-particles predicted as they are
 * loaded), then one workgroup per cluster for the corrector, the new levels and the next
 * block.  A run replays a HIP
 * graph of steps_per_launch global steps until every cluster is done.
 * The state is one nb_state over all particles, clusters stored contiguously.
 * ------------------------------------------------------------------------------------------ */
typedef struct nb_ens nb_ens;

/* Create an ensemble of n_clusters clusters: cluster c holds particles [offsets[c],
 * offsets[c+1]) (HOST array of n_clusters + 1, offsets[0] = 0, strictly increasing, total
 * <= 2^28, n_clusters <= 8192) with softening eps[c] > 0 (HOST array); steps in
 * [2^-lmax, 2^-lmin]; interaction arithmetic `precision` (NB_FP32, NB_DS or NB_FP64).
 * Allocates no device memory (see nb_ens_bind_scratch). */
nb_status nb_ens_create(nb_ens **out, int32_t n_clusters, const int32_t *offsets,
                        const double *eps, int32_t lmin, int32_t lmax, int32_t precision);

/* Bytes of device workspace an ensemble of these clusters needs (offsets as for
 * nb_ens_create, HOST array): cluster tables, per-cluster records, block lists, criterion and
 * energy scratch, and one plane set of j-split partial sums per cluster (7 doubles per
 * particle per 256-particle j-tile).  0 if the arguments are invalid. */
size_t nb_ens_scratch_bytes(int32_t n_clusters, const int32_t *offsets, int32_t precision);

/* Bind the ensemble's workspace (as nb_bind_scratch: caller-owned, 256-byte aligned, at least
 * nb_ens_scratch_bytes() bytes); uploads the cluster tables.  Synchronising.  Required before
 * nb_ens_init. */
nb_status nb_ens_bind_scratch(nb_ens *ens, void *scratch, size_t bytes);

/* Release the ensemble (never the caller's memory).  NULL is a no-op. */
nb_status nb_ens_destroy(nb_ens *ens);

/* Enqueue subsequent work on `hip_stream` (NULL: the null stream). */
nb_status nb_ens_set_stream(nb_ens *ens, void *hip_stream);

/* Bind the caller's FP64 state over all particles (as nb_bind). */
nb_status nb_ens_bind(nb_ens *ens, const nb_state *state);

/* Force work layout (the autotuner's knobs): whole 256-particle j-tiles per work item for
 * each cluster (HOST array of n_clusters values >= 1, or NULL to keep; default: the fewest
 * that leave each cluster at most 4 j-ranges, so its own workgroup sums at most 4 partial
 * planes per block particle), i-particles per work-item (must be 1: block particles instead
 * share lanes, nb_ens_set_split) and j-loop unroll (1 or 2, default 2).  Synchronising. */
nb_status nb_ens_set_layout(nb_ens *ens, const int32_t *tiles_per_item, int32_t ipl,
                            int32_t unroll);

/* Which blocks each cluster's own workgroup advances: a selected block of n_act <= 1024
 * particles with n_act * N_c <= local_limit interactions (0: none) is forced, corrected and
 * followed by the cluster's next block inside the cluster's workgroup (all its particles
 * predicted as they are staged in LDS), up to local_steps such block steps and local_work
 * interactions per cluster per global step; larger blocks go through the GPU-wide force of the
 * next global step.  Only the summation order differs between the two paths.  Defaults: 0
 * (every block through the GPU-wide force), 64, 2^21.  Synchronising. */
nb_status nb_ens_set_local(nb_ens *ens, int64_t local_limit, int32_t local_steps,
                           int64_t local_work);

/* Independent lanes: lane_of (HOST array of n_clusters values in [0, lanes); NULL allowed
 * when lanes == 1) assigns every cluster to one of `lanes` groups (1 to 3, each non-empty;
 * default 1).  nb_ens_run then advances each lane by global steps of its own clusters only, its
 * graph replayed on a stream of its own (created by the library at the default priority), so a
 * lane whose clusters need few block steps is not held to the step count of another, and one
 * lane's kernels overlap another's.  The clusters are independent, so every result is bitwise
 * the same for any assignment; work queued later on the ensemble's stream waits for all lanes.
 * The assignment that pays is one that gives the clusters with the most block steps a lane of
 * their own.  NB_EINVAL otherwise.  Synchronising. */
nb_status nb_ens_set_lanes(nb_ens *ens, int32_t lanes, const int32_t *lane_of);

/* Force work-item size (an autotuner knob): every block particle of a force item is shared by
 * at least smin lanes (a power of two in [1, 64]; default 8), each taking every smin-th j of a
 * tile, so an item holds at most 256 / smin block particles.  Smaller items balance a global
 * step whose clusters' blocks differ in size by orders of magnitude; the sums combine the
 * lanes' parts by wave shuffles in a fixed order.  NB_EINVAL otherwise.  Synchronising. */
nb_status nb_ens_set_split(nb_ens *ens, int32_t smin);

/* Sec. 2 start of run for every cluster: full force at time 0, initial steps from
 * Eq. initTimestep with this eta, times 0. */
nb_status nb_ens_init(nb_ens *ens, double eta);

/* Advance every cluster by its own block steps until its next block would pass t_end
 * (ticks), steps_per_launch global steps per graph launch (use_graph != 0) or eager launch
 * batch, synchronising after each to test for completion; at most max_steps global steps
 * (<= 0: no limit).  A global step is the GPU-wide force of every cluster's selected block that
 * is not a local block (nb_ens_set_local), then one workgroup per cluster: the corrector of
 * that block, the next block, and the cluster's local block steps.  Returns NB_OK or a latched
 * device error. */
nb_status nb_ens_run(nb_ens *ens, double eta, int64_t t_end, int32_t steps_per_launch,
                     int64_t max_steps, int32_t use_graph);

/* Per-cluster scheduler records into the HOST array out[n_clusters] (flags = 1 once the
 * cluster has reached t_end).  Synchronising. */
nb_status nb_ens_control(nb_ens *ens, nb_control *out);

/* Sec. 4.2 energy of every cluster at its current time, FP64 (HOST arrays of n_clusters).
 * Synchronising. */
nb_status nb_ens_energy(nb_ens *ens, double *ekin, double *epot);

/* Message for the last failing call on an ensemble (never NULL). */
const char *nb_ens_last_error(const nb_ens *ens);

/* Human-readable message for the last failing call on ctx (never NULL). */
const char *nb_last_error(const nb_ctx *ctx);

/* Library version string, e.g. "libnbody 0.1 gfx950". */
const char *nb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NBODY_H */
