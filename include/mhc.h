/*
 * mhc.h -- C ABI of the MI355X multi-hypothesis criticality library.
 *
 * The library evaluates the data-parallel core of the multi-hypothesis
 * criticality method of Sanchez Morales et al., "Parallel Multi-Hypothesis
 * Algorithm for Criticality Estimation in Traffic and Collision Avoidance"
 * (IEEE IV 2019): it generates a grid of trajectory hypotheses per object
 * (Sec. III, Sec. IV-B), tests every pair of predicted poses of every pair of
 * objects at every time step for overlap (Sec. IV-C), keeps the earliest
 * colliding step of each trajectory pair, and reduces those to a criticality
 * per trajectory and per object (Sec. IV-D). A scene goes in, criticalities
 * come out (the paper's input / output boxes of Fig. 1, Sec. V).
 *
 * Conventions shared by every entry point
 *   - All functions return an mhc_status; negative values are errors and
 *     mhc_last_error(ctx) then holds a message owned by the context, valid
 *     until the next call on that context. No C++ exception crosses the ABI.
 *   - Inputs are validated before anything is launched; on an error no output
 *     buffer is written.
 *   - The caller owns every buffer passed in. Scenes are copied during the
 *     call (mhc_submit copies before it returns), so they may be freed after.
 *   - A context is used by one thread at a time. Server calls (mhc_submit,
 *     mhc_wait, mhc_server_stats) are thread-safe.
 *   - Units are SI (m, s, rad); doubles in, doubles out. GPU arithmetic is
 *     FP64 for trajectories and probabilities and FP32 for the overlap tests.
 *     Before the FP32 poses are stored, every position is taken relative to
 *     a per-scene origin (the middle of the box of the initial positions,
 *     rounded to a multiple of 256 m), so a scene far from (0, 0) is tested
 *     as precisely as one near it. First hits agree with an exact FP64
 *     evaluation wherever the overlap margin exceeds 1e-4 m while the poses
 *     stay within about 256 m of that origin; further out the FP32 rounding
 *     of the tests grows in proportion to the distance.
 *   - Time slots: slot t in [0, horizon) is the pose predicted for time
 *     (t+1)*dt; the measured state at time 0 is never tested.
 */
#ifndef MHC_H
#define MHC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mhc_ctx mhc_ctx;
typedef struct mhc_plan mhc_plan;
typedef struct mhc_server mhc_server;

typedef enum {
    MHC_OK = 0,
    MHC_E_INVAL = -1,    /* malformed input: nothing launched, outputs untouched */
    MHC_E_NOMEM = -2,    /* host or device allocation failed / budget exceeded */
    MHC_E_DEVICE = -3,   /* no usable GPU, or a HIP call failed */
    MHC_E_BUSY = -4,     /* server queue full; retry later */
    MHC_E_TIMEOUT = -5   /* mhc_wait timed out; the ticket stays valid */
} mhc_status;

enum { MHC_VEHICLE = 0, MHC_PEDESTRIAN = 1 };
/* Pair set: every unordered object pair, or only pairs with the EGO vehicle
 * (object 0) as in Sec. IV-C.1, where combinations between collision objects
 * are left out. */
enum { MHC_PAIRS_ALL = 0, MHC_PAIRS_EGO = 1 };
/* Overlap test of the collision recognition (Sec. IV-C.1).
 * EXACT: the closed shapes intersect (rectangle-rectangle by separating axes,
 *   rectangle-circle and circle-circle by exact distances).
 * PIP: the paper's own test, a point-in-polygon check of every vertex of each
 *   object's polygon against the other object's polygon, in both directions.
 *   Every object must be a vehicle (rectangle); a vertex on the other
 *   rectangle's boundary counts as inside. It misses overlaps in which no
 *   vertex of either lies inside the other (two bars crossing). */
enum { MHC_OVERLAP_EXACT = 0, MHC_OVERLAP_PIP = 1 };
/* Reading of the conditional-probability approximation (Sec. IV-D.2): how
 * the colliding combinations of one trajectory of object a with the
 * trajectories j of another object b make up the probability q_{a,i;b} that
 * the collision with b happens.
 * EXCLUSIVE: b follows exactly one of its trajectories, so the colliding
 *   ones add up: q = sum_j [hit] p_{b,j} (with one collision object this is
 *   the paper's p_cra double sum of Sec. IV-D).
 * INDEPENDENT: every combination is an independent event, scaled by the
 *   no-collision probability of the ones before it:
 *   q = 1 - prod_j (1 - [hit] p_{b,j}).
 * In both readings collision objects are independent of one another and
 * crit_{a,i} = 1 - prod_{b != a} (1 - q_{a,i;b}). */
enum { MHC_RISK_EXCLUSIVE = 0, MHC_RISK_INDEPENDENT = 1 };

/* One traffic participant. Vehicles are rectangles (length along the heading,
 * width across it) moving on the kinematic special case of the Euler pose
 * update of Sec. IV-B.1 (side slip 0) under a constant acceleration u[k] and
 * yaw rate w[l]; the speed is clamped at 0. Pedestrians are circles of radius
 * `radius` walking at constant speed u[k] along heading + w[l] (Sec. IV-B.3).
 * Trajectory i = k*n_w + l. `score` holds n_u*n_w non-negative scores that are
 * L1-normalised into probabilities (Sec. IV-D.1); NULL means uniform.
 * A vehicle may instead be a general convex polygon (Sec. IV-C.1 allows
 * polygons of any complexity): `vertices` holds n_vertices
 * (x, y) pairs in the body frame (x along the heading, y to the left, origin
 * at the tracked position), 3 <= n_vertices <= MHC_MAX_VERTICES, strictly
 * convex, counter-clockwise, every interior angle at least 45 degrees;
 * length and width are then ignored. A pair with such an outline is tested
 * polygon against polygon (a rectangle by its four corners) or polygon
 * against circle, in either overlap mode. */
enum { MHC_MAX_VERTICES = 8 };
/* Motion model of an object's trajectory grid (Sec. IV-B).
 * KINEMATIC (0, default): as described above.
 * PED_ACCEL (1, pedestrians, Sec. IV-B.3): u[k] constant accelerations,
 *   w[l] absolute headings; the speed follows v_{n+1} = v_n + a tau, the
 *   acceleration of a step cut so that 0 <= v_{n+1} <= params[0] (v_max,
 *   2.7 m/s in the paper), the position the Euler update of the paper.
 * ONE_TRACK (2, vehicles, Sec. IV-B.1): the linear one-track model with
 *   params = {c_alpha_f, c_alpha_r [N/rad], l_f, l_r [m], m [kg], I_z
 *   [kg m^2]} (all > 0, understeer: l_r c_alpha_r >= l_f c_alpha_f), u[k]
 *   constant accelerations (speed stopping at 0), w[l] constant front
 *   steering angles [rad]; side slip and yaw rate start at 0 and follow the
 *   model's Euler update, except that where that explicit step is unstable
 *   (low speed: an eigenvalue of I + tau A(v) of modulus >= 1) they take the
 *   model's steady state at the new speed. */
enum { MHC_MODEL_KINEMATIC = 0, MHC_MODEL_PED_ACCEL = 1, MHC_MODEL_ONE_TRACK = 2 };
typedef struct {
    int32_t kind;                 /* MHC_VEHICLE or MHC_PEDESTRIAN */
    double x, y, heading, speed;  /* measured state at time 0; speed >= 0 */
    double length, width;         /* vehicles without an outline: full extents > 0 */
    double radius;                /* pedestrians: > 0 (ignored for vehicles) */
    int32_t n_u, n_w;             /* grid sizes, >= 1 each */
    const double *u, *w;          /* n_u and n_w finite control values */
    const double *score;          /* n_u*n_w scores or NULL */
    int32_t n_vertices;           /* 0 (rectangle / circle) or 3..MHC_MAX_VERTICES (vehicles) */
    const double *vertices;       /* 2*n_vertices body-frame coordinates x0, y0, x1, y1, ... */
    int32_t model;                /* MHC_MODEL_* motion model of the trajectory grid */
    double params[6];             /* parameters of the motion model (see MHC_MODEL_*) */
} mhc_object;

typedef struct {
    int32_t n_objects;            /* >= 2; object 0 is the EGO vehicle */
    const mhc_object *objects;
    int32_t horizon;              /* steps H, 1..32767 */
    double dt;                    /* step length tau > 0 */
    int32_t pairs;                /* MHC_PAIRS_ALL or MHC_PAIRS_EGO */
    int32_t overlap;              /* MHC_OVERLAP_EXACT or MHC_OVERLAP_PIP */
    int32_t risk;                 /* MHC_RISK_EXCLUSIVE or MHC_RISK_INDEPENDENT */
    int32_t timeline;             /* 1: also the criticality over time and its
                                     attribution (crit_t ... traj_attrib below) */
} mhc_scene;

typedef struct {
    int64_t n_traj;               /* sum_a T_a */
    int64_t n_pairs;              /* object pairs evaluated */
    int64_t n_traj_pairs;         /* sum over pairs T_a*T_b (first-hit entries) */
    int64_t n_checks;             /* n_traj_pairs * horizon pose-pair checks */
    size_t device_bytes;          /* workspace bytes mhc_evaluate_async needs */
} mhc_sizes;

/* Outputs. Host pointers for mhc_evaluate / mhc_evaluate_batch / mhc_submit,
 * device pointers for mhc_evaluate_async / mhc_plan_execute. Any pointer but
 * object_crit may be NULL.
 *   object_crit [n_objects]      C_a = sum_i p_{a,i} crit_{a,i}
 *   traj_crit   [n_traj]         crit_{a,i} = 1 - prod_{b != a} (1 - q_{a,i;b})
 *   traj_prob   [n_traj]         p_{a,i}, the normalised scores
 *   q           [n_traj*n_objects] q_{a,i;b} (see MHC_RISK_*); 0 for b == a
 *                                  and for pairs outside the pair set
 *   first_hit   [n_traj_pairs]   per pair (a < b, lexicographic), entry i*T_b + j:
 *                                  earliest colliding slot, or -1
 * Trajectories of object a start at index sum_{c<a} T_c. With a single
 * collision object C_0 equals the paper's p_cra double sum (Sec. IV-D); with
 * several, the chronological scaling of Sec. IV-D.2 is applied, collision
 * objects being independent.
 *
 * Over time (only for scenes with `timeline` = 1; must be NULL otherwise).
 * The colliding combinations of trajectory (a, i) are taken in the order of
 * their first colliding slot (ties: ascending object, then trajectory index);
 * each counts with its probability scaled by the probability that no
 * collision happened before it (Sec. IV-D.2):
 *   crit_t      [n_objects*horizon]  C_a(s) = sum_i p_{a,i} crit_{a,i}(s), the
 *                                  probability of a collision of a at or
 *                                  before slot s (time (s+1)*dt); the rise of
 *                                  C over the horizon is what the anticipation
 *                                  time of Sec. IV-D / VI-A is read from
 *   traj_crit_t [n_traj*horizon]     crit_{a,i}(s), entry (i, s) at i*horizon + s
 *   attrib      [n_objects*n_objects] A_{a,b} = sum_i p_{a,i} A_{a,i;b}, the
 *                                  probability that a's first collision is
 *                                  with b; sum_b A_{a,b} = C_a
 *   traj_attrib [n_traj*n_objects]   A_{a,i;b}, entry (i, b) like q
 * crit_t at slot horizon-1 and sum_b attrib equal object_crit up to rounding
 * (they are summed in another order). */
typedef struct {
    double *object_crit;
    double *traj_crit;
    double *traj_prob;
    double *q;
    int16_t *first_hit;
    double *crit_t;
    double *traj_crit_t;
    double *attrib;
    double *traj_attrib;
} mhc_result;

/* ---- context ---------------------------------------------------------- */

/* System entry point with no passage of its own (the paper's module chain,
 * Fig. 1, runs inside the calls below). Opens GPU `device` and reserves no
 * workspace yet (the allocation-free entry point's device array is located
 * here). hbm_budget_bytes caps the device memory the context (and a server
 * started on it) may hold; 0 means no cap. Returns MHC_E_INVAL for a NULL
 * `out` or a device index out of range, MHC_E_DEVICE when no gfx950 GPU is
 * usable; *out is NULL on error. mhc_destroy waits for the context's work and
 * frees it (NULL is ignored). */
mhc_status mhc_create(int device, size_t hbm_budget_bytes, mhc_ctx **out);
void mhc_destroy(mhc_ctx *ctx);
const char *mhc_last_error(const mhc_ctx *ctx);

/* Host only (no GPU needed): validates `scene` and reports its sizes.
 * The trajectory count corresponds to r_tra of Sec. IV-B.4 and n_traj_pairs to
 * r_col of Sec. IV-C.2 in the EGO pair mode. */
mhc_status mhc_query_sizes(const mhc_scene *scene, mhc_sizes *out);

/* Host only (no GPU needed). Anticipation time (Sec. IV-D, Sec. VI-A): how
 * long before an event the criticality of a situation is recognised.
 * crit[f] is the criticality of frame f of an evolving scene, frames
 * frame_dt seconds apart (for instance object_crit[0] of successive
 * evaluations); the event (the collision) happens at frame event_frame,
 * 1 <= event_frame <= n_frames. The criticality counts as recognised from the
 * first frame f* from which crit[g] >= threshold for every g in
 * [f*, event_frame); *out_seconds = (event_frame - f*) * frame_dt, and 0 when
 * crit[event_frame - 1] < threshold. MHC_E_INVAL for NULL pointers, a frame
 * index out of range, frame_dt <= 0, or a non-finite threshold or crit. */
mhc_status mhc_anticipation_time(int32_t n_frames, const double *crit, double frame_dt, double threshold,
                                 int32_t event_frame, double *out_seconds);

/* ---- plain single scene ------------------------------------------------ */

/* Synchronous: host scene in, host results out. Runs ingest (validation,
 * pair list, work list), trajectory generation, collision recognition and
 * risk assessment (Fig. 1) and returns when the results are in `res`. */
mhc_status mhc_evaluate(mhc_ctx *ctx, const mhc_scene *scene, mhc_result *res);

/* The path of Fig. 1 as mhc_evaluate (Sec. IV-B to IV-D), enqueued
 * asynchronously on the caller's HIP stream (`hip_stream`, a hipStream_t; NULL
 * is the null stream) with caller-owned device memory: `dev_workspace` of at
 * least mhc_query_sizes().device_bytes bytes (256-byte aligned) and the device
 * pointers in `dev_out`. The scene is validated and packed on the host and
 * copied into the workspace by an asynchronous copy on that stream; nothing
 * is freed or synchronised. The workspace and outputs must stay valid until
 * the stream passes this work. */
mhc_status mhc_evaluate_async(mhc_ctx *ctx, const mhc_scene *scene, void *dev_workspace,
                              size_t workspace_bytes, const mhc_result *dev_out, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * work as mhc_evaluate_async, with the workspace in a library-owned device
 * array of MHC_NOALLOC_MAX_BYTES bytes instead of caller memory. The array
 * is a file-scope device variable: every GPU the library runs on holds one
 * copy of it until the process ends, and its address is looked up once per
 * device in mhc_create. The call allocates no device or pinned host memory
 * (the host tables of the scene reuse the context's storage) and frees
 * nothing; the scene image goes up from pageable host memory on `hip_stream`.
 * `dev_out` holds device pointers as for mhc_evaluate_async (object_crit
 * required; outputs left NULL stay in the array). Whatever must start at zero
 * (the q accumulators, the risk kernel's counters, the per-slot sums) is
 * cleared by the trajectory kernel of the same call.
 * Errors: MHC_E_INVAL as mhc_evaluate_async; MHC_E_NOMEM when the scene's
 * workspace exceeds MHC_NOALLOC_MAX_BYTES (nothing is launched).
 * All calls on one GPU share its array and it keeps the last call's contents:
 * calls whose work overlaps on the device (other streams, other contexts or
 * threads on the same GPU) race and give undefined results; calls on one
 * stream are ordered. Results equal mhc_evaluate_async bit for bit. */
enum { MHC_NOALLOC_MAX_BYTES = 64 << 20 };
mhc_status mhc_evaluate_noalloc(mhc_ctx *ctx, const mhc_scene *scene, const mhc_result *dev_out, void *hip_stream);

/* ---- device-resident plan ---------------------------------------------- */

/* Validates `scene`, builds its pair and work lists on the host and uploads
 * the raw inputs (states, control grids, scores) to device memory owned by
 * the plan. mhc_plan_execute then runs the whole device path -- probability
 * normalisation, trajectory generation, collision recognition, risk -- on
 * those resident inputs; it can be called any number of times.
 * mhc_plan_update replaces the values of a scene with the same shape (object
 * kinds, grid sizes, horizon, pair mode) without rebuilding the lists. */
mhc_status mhc_plan_create(mhc_ctx *ctx, const mhc_scene *scene, mhc_plan **out);
mhc_status mhc_plan_update(mhc_plan *plan, const mhc_scene *scene);
/* Launches on `hip_stream`. Device pointers in `dev_out` (NULL entries are
 * kept in plan-owned memory). */
mhc_status mhc_plan_execute(mhc_plan *plan, const mhc_result *dev_out, void *hip_stream);
/* The same work split by module (Fig. 1): any combination of the stage bits,
 * launched in module order on `hip_stream`. Lets a caller time or interleave
 * the modules; a stage reads what the previous stages of an earlier or the
 * same call left in the plan's (or dev_out's) buffers. */
enum { MHC_STAGE_TRAJ = 1, MHC_STAGE_COLLIDE = 2, MHC_STAGE_RISK = 4, MHC_STAGE_ALL = 7 };
mhc_status mhc_plan_execute_stages(mhc_plan *plan, const mhc_result *dev_out, void *hip_stream,
                                   uint32_t stages);
/* Launch mode of mhc_plan_execute: 0 (default) enqueues the module kernels
 * directly; 1 captures them once per set of output pointers into a HIP graph
 * and replays it (one launch call; results identical). */
mhc_status mhc_plan_set_graph(mhc_plan *plan, int32_t enable);
/* Copies the plan-owned results of the last execute to host buffers (sync). */
mhc_status mhc_plan_download(mhc_plan *plan, mhc_result *host_out);
void mhc_plan_destroy(mhc_plan *plan);

/* ---- collision-kernel tile shapes (autotuning) --------------------------- */

/* The collision kernel is compiled for MHC_N_VARIANTS micro-tile shapes (how
 * many trajectories of each object one GPU thread pairs up). Results are
 * bit-identical for every variant; only speed differs.
 * mhc_set_variant forces one (-1 returns to the tuned choice).
 * mhc_autotune times every variant on `scene` in interleaved passes (the
 * variants in turn, two collision launches back to back each, every variant
 * on an image of its own when all fit in device memory, else one variant at
 * a time): a warm-up pass, `reps` timed passes, and further passes while
 * the fastest variant's median over the last `reps` passes still falls by
 * more than 1 % (a GPU coming out of idle raises its clock over the first
 * milliseconds), up to 20 reps passes or 0.5 s. It records the fastest for
 * scenes of the same size class: log2 buckets of the mean trajectory count
 * per object and of the mean horizon, the test family (0 rectangles and
 * circles, 1 point-in-polygon rectangles, 2 outlines) and a log2 bucket of
 * the scene count (0 for one scene). `us` (or NULL) receives each variant's
 * median microseconds per collision launch over the last `reps` passes
 * (host array of MHC_N_VARIANTS). reps in [1, 100000], else MHC_E_INVAL.
 * mhc_autotune_batch does the same for n scenes evaluated together
 * as mhc_evaluate_batch launches them (one collision launch for all), so
 * batches of that class use the variant found fastest for the batch; errors
 * as mhc_evaluate_batch (the tuned choices are left unchanged on error).
 * mhc_tune_save / mhc_tune_load write / read the recorded choices as JSON
 * ({"gfx950": {"<T bucket>,<H bucket>,<family>,<scenes bucket>": variant,
 * ...}}; keys with two or three fields, from earlier files, are read with
 * the missing fields 0). A file that cannot be read, has no "gfx950" object
 * or holds an entry that does not parse or names a variant outside
 * [0, MHC_N_VARIANTS) gives MHC_E_INVAL and changes nothing. */
enum { MHC_N_VARIANTS = 4 };
mhc_status mhc_set_variant(mhc_ctx *ctx, int32_t variant);
mhc_status mhc_autotune(mhc_ctx *ctx, const mhc_scene *scene, int32_t reps, int32_t *best_variant, double *us);
mhc_status mhc_autotune_batch(mhc_ctx *ctx, int32_t n, const mhc_scene *scenes, int32_t reps, int32_t *best_variant,
                              double *us);
mhc_status mhc_tune_save(mhc_ctx *ctx, const char *path);
mhc_status mhc_tune_load(mhc_ctx *ctx, const char *path);

/* ---- collision plan check (host only) ----------------------------------- */

/* The collision work of n scenes is cut into units (a wave's items of one
 * object pair: row-major runs of the pair's item grid, or 2-D blocks of it)
 * that the host deals to the waves of the collision kernel (Sec. IV-C: every
 * trajectory of one object against every trajectory of another, at every
 * step). mhc_plan_check builds the plan the library would launch for tile
 * variant `variant` (0 .. MHC_N_VARIANTS-1) with `max_waves` resident waves
 * (0: one wave per unit) and walks it on the host the way the kernel decodes
 * it. It needs no GPU. MHC_OK when every trajectory pair of every object pair
 * is tested by exactly one thread and every index a thread derives (items,
 * trajectories, steps, first-hit entries) lies inside its pair; MHC_E_INVAL
 * for an invalid scene or argument (info untouched) or a plan that fails the
 * check (info filled). */
typedef struct {
    int64_t n_units;        /* collision units of the plan */
    int64_t n_waves;        /* wave slots the units are dealt to */
    int64_t blocked_pairs;  /* object pairs whose units are 2-D blocks of items */
    int64_t uncovered;      /* items tested by no thread (0 when the plan is sound) */
    int64_t repeated;       /* items tested more than once (0 when sound) */
    int64_t out_of_range;   /* threads deriving an index outside their pair (0 when sound) */
    int32_t contiguous;     /* 1: waves take contiguous stretches of the unit sequence */
    int32_t time_split;     /* largest number of step ranges a unit is cut into (1, 2, 4 or 8) */
} mhc_plan_info;
mhc_status mhc_plan_check(int32_t n_scenes, const mhc_scene *scenes, int32_t variant, int32_t max_waves,
                          mhc_plan_info *info);

/* ---- batched ----------------------------------------------------------- */

/* A system form with no passage of its own: the path of Fig. 1 for n scenes
 * of any shapes at once, one trajectory launch, one collision launch and one
 * risk launch for all of them (captured as a HIP graph when the batch's shape
 * key comes back), then every result copied to res[k] (host buffers; any
 * field but object_crit may be NULL per scene). Results are identical to
 * mhc_evaluate of each scene alone. MHC_E_INVAL for n < 1, NULL arrays, an
 * invalid scene or result set (the message names the scene index) or more
 * than 65535 objects in all; MHC_E_NOMEM / MHC_E_DEVICE as mhc_evaluate;
 * on error no output is written. */
mhc_status mhc_evaluate_batch(mhc_ctx *ctx, int32_t n, const mhc_scene *scenes, mhc_result *res);

/* ---- served (continuous batching) ------------------------------------- */

/* A system form with no passage of its own in the paper: the request loop
 * around the module chain of Fig. 1 (the paper's own I/O layer, Sec. V,
 * serves one request at a time). Frames from many streams are admitted into
 * "ticks" (one batched evaluation each) while earlier ticks still run. */
typedef struct {
    size_t hbm_budget_bytes;      /* device bytes the server may hold for frames; 0 = ctx budget or 1 GiB;
                                     each of the max_inflight_ticks slots gets an equal share */
    int32_t max_inflight_ticks;   /* ticks running at once (1..4; 0 = 2) */
    int32_t queue_capacity;       /* frames waiting for admission (0 = 4096) */
    int32_t max_frames_per_tick;  /* 0 = 256 */
    int64_t max_checks_per_tick;  /* a tick closes when this many checks are admitted (0 = 4e9); a frame
                                     of more checks rides in a tick of its own, its collision work cut
                                     into launches of at most about this many checks so that other
                                     ticks reach the GPU in between; with two or more slots such frames
                                     hold all but one slot, so one slot stays open to smaller frames
                                     (which may then overtake a waiting large one) */
    int64_t watchdog_us;          /* a tick running longer than this fails the server: its frames and
                                     every queued one complete with MHC_E_DEVICE, mhc_server_stop
                                     returns MHC_E_DEVICE (0 = 30 s) */
    int64_t deadline_us;          /* frames slower than this (submit -> results) count as late in
                                     mhc_stats (0 = no deadline) */
} mhc_server_cfg;

typedef struct {
    int64_t submit_ns, admit_ns, launch_ns, done_ns;  /* monotonic clock (CLOCK_MONOTONIC), ns */
    int64_t tick;                 /* tick that carried the frame */
} mhc_timing;

typedef struct {
    int64_t submitted, completed, rejected, deferred;  /* deferred = ticks that left frames queued */
    int64_t ticks, checks;
    int64_t late;                 /* completed frames over deadline_us */
    double p50_ms, p99_ms, max_ms, mean_ms;            /* submit -> results in host memory */
    double checks_per_s;          /* completed checks / wall time since start */
} mhc_stats;

/* Starts a scheduler thread on the GPU of `ctx`. Frames submitted from any
 * thread are admitted, in arrival order, into the next tick while their
 * device memory fits the slot's budget; ticks run on separate streams so that
 * a new tick is built and launched while earlier ones are still on the GPU.
 * The context's tile-variant choices (mhc_set_variant, mhc_autotune, tune
 * files) are copied at start; later changes to them do not reach a running
 * server, and the context stays usable by its own thread meanwhile. */
mhc_status mhc_server_start(mhc_ctx *ctx, const mhc_server_cfg *cfg, mhc_server **out);
/* Copies `scene` and queues it; `dst` (host buffers) receives the results and
 * must stay valid until mhc_wait reports completion. MHC_E_INVAL for an
 * invalid scene or result set (or a stopping server), MHC_E_BUSY when the
 * queue is full, MHC_E_NOMEM when the frame can never fit a slot's budget. */
mhc_status mhc_submit(mhc_server *srv, int32_t stream_id, const mhc_scene *scene, mhc_result *dst,
                      uint64_t *ticket);
/* Waits up to timeout_us (< 0: forever) for `ticket`; fills `timing` if not
 * NULL. A ticket can be waited on once successfully; the frame's status
 * (MHC_OK, or MHC_E_DEVICE when its tick failed) is returned. MHC_E_TIMEOUT
 * leaves the ticket valid; an unknown ticket gives MHC_E_INVAL. */
mhc_status mhc_wait(mhc_server *srv, uint64_t ticket, int64_t timeout_us, mhc_timing *timing);
mhc_status mhc_server_stats(mhc_server *srv, mhc_stats *out);
/* Drains running ticks, completes queued frames, joins the thread, frees.
 * MHC_E_DEVICE when a tick failed or tripped the watchdog while it ran. */
mhc_status mhc_server_stop(mhc_server *srv);

/* A tick executor supplied by the caller, for running the scheduler without
 * the library's GPU path (tests of admission, ordering, deadlines and the
 * watchdog; other devices). Called from the scheduler thread only.
 *   launch: start tick `tick` in slot `slot` (0 .. max_inflight_ticks-1) with
 *           n frames, their scenes and host result buffers (valid until the
 *           tick is reported done); return MHC_OK or a negative mhc_status
 *           (the tick's frames then fail with MHC_E_DEVICE).
 *   poll:   1 when the slot's tick has finished and its results are in the
 *           buffers, 0 while it runs, < 0 when it failed.
 * mhc_server_start_executor copies *ex; the server has no context (budgets
 * as in cfg, default 1 GiB). MHC_E_INVAL for a NULL argument or callback or
 * a configuration out of range. */
typedef struct {
    void *user;
    int32_t (*launch)(void *user, int32_t slot, int64_t tick, int32_t n_frames, const mhc_scene *scenes,
                      const mhc_result *dsts);
    int32_t (*poll)(void *user, int32_t slot);
} mhc_executor;
mhc_status mhc_server_start_executor(const mhc_server_cfg *cfg, const mhc_executor *ex, mhc_server **out);

#ifdef __cplusplus
}
#endif
#endif /* MHC_H */
