/*
 * mppi.h -- C ABI of libmppi.so, an MI355X (gfx950) implementation of the
 * hot path of torque-sampling MPPI with analytic rigid-body dynamics
 * (Im et al., "Real-Time Dynamics-Based Torque-Sampling MPPI for Compliant
 * and Force Aware Manipulation").
 *
 * One update (Sec. II Eqs. 1-4 and Sec. III):
 *   - K perturbed torque sequences v_k,t = u_t + du_k,t (Eq. 2, Sec. III-A
 *     "torque-level sampling"), du drawn per (tick, sample, step, joint)
 *     from Philox4x32-10 + Box-Muller;
 *   - each rolled out for T steps through 7-DoF forward dynamics (Eqs. 5-6;
 *     on the default launch shape from composite-rigid-body inertias and an
 *     LDL^T solve with eight lanes per sample, on the per-lane shapes and in
 *     batches by the articulated-body algorithm, see mppi_set_launch) and
 *     the semi-implicit Euler step written in Eq. 7;
 *   - the running cost of Eqs. 9-14 (EE position/orientation, dynamically
 *     consistent EE force, joint/torque limit penalties) at every step and
 *     a terminal cost phi(x_T) (Eq. 3);
 *   - importance weights with the minimum-cost shift (Eq. 4a and the text
 *     after it) and the weighted noise average that updates the nominal
 *     sequence (Eq. 4b).
 *
 * Conventions: all host-side structs are FP64; matrices row-major;
 * frames and joint model as documented at mppi_link_params; task-space
 * wrenches ordered [force; moment] and world-aligned.  Every call returns
 * an mppi_status code; no call throws, aborts or prints.
 *
 * Threading: a handle may be used from one host thread at a time.  Calls
 * that take a stream enqueue work and return; the caller synchronises.
 */
#ifndef MPPI_H
#define MPPI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPPI_NJ 7 /* joints supported by the kernels */
#define MPPI_MAX_OBSTACLES 4
#define MPPI_MAX_PAIRS 32
#define MPPI_MAX_ITERATIONS 64

typedef enum {
    MPPI_OK = 0,
    MPPI_EINVAL = 1,      /* bad argument (null, size, non-finite, range) */
    MPPI_ENONFINITE = 2,  /* every sample cost was non-finite: U_new = U_nominal */
    MPPI_ENOMEM = 3,      /* device or pinned host allocation failed */
    MPPI_EDEVICE = 4,     /* a HIP runtime call or kernel launch failed */
    MPPI_ENOTSUP = 5,     /* valid request this build does not implement */
    MPPI_ESCRATCH = 6     /* mppi_update_noalloc: needs more than its static workspace */
} mppi_status;

typedef enum { MPPI_FP32 = 0, MPPI_FP64 = 1 } mppi_precision;
/* Forward dynamics of the rollouts: MPPI_DYN_ABA (default) is the
 * recursive route (the articulated-body algorithm on the per-lane launch
 * shapes and in batches; on the eight-lane launch shape the same
 * quantities from composite-rigid-body inertias and an LDL^T solve), or
 * the paper's own route, M formed by the Jacobian sum of Eq. 8 and h from
 * the Jacobian time derivatives, solved by Cholesky. */
typedef enum { MPPI_DYN_ABA = 0, MPPI_DYN_EXPLICIT_M = 1 } mppi_dynamics;
typedef enum { MPPI_EXT_NONE = 0, MPPI_EXT_CONST = 1, MPPI_EXT_WALL = 2 } mppi_ext_mode;

/* One link of the serial chain (Fig. 1 caption: joint transforms and CoM
 * offsets per link).  Frame i relative to frame i-1: origin r_parent,
 * orientation R_parent * Rz(q_i); joint i rotates about its local z. */
typedef struct {
    double R_parent[9];   /* row-major rotation, frame i-1 axes */
    double r_parent[3];   /* [m], frame i-1 axes */
    double mass;          /* [kg], > 0 */
    double com[3];        /* CoM in frame i [m] */
    double inertia_com[6];/* about the CoM, frame-i axes: xx yy zz xy xz yz; PD,
                             triangle inequality (Eq. 8's I^G rotated into frame i) */
    double armature;      /* >= 0, the diag(a) term of Eq. 8 [kg m^2] */
    double q_min, q_max;  /* [rad] */
    double qd_max;        /* [rad/s] */
    double tau_max;       /* [N m] */
} mppi_link_params;

typedef struct {
    int n_joints;                    /* must be MPPI_NJ */
    mppi_link_params link[MPPI_NJ];
    double R_ee[9];                  /* EE frame in the last link frame */
    double r_ee[3];                  /* EE point in the last link frame [m] */
    double gravity[3];               /* world gravity [m/s^2], e.g. 0 0 -9.81 */
} mppi_robot_params;

/* Cost and sampler settings.  Weights are the diagonals of Eqs. 11-12
 * (axis selection); C_joint uses squared hinges on the limits plus a
 * posture term; C_torque penalises |v_j| beyond tau_max with a squared
 * hinge; phi(x_T) = w_terminal * (C_pos + C_ori + C_joint)(x_T). */
typedef struct {
    int K;                   /* samples, 1 .. 1<<20 */
    int T;                   /* horizon steps, 1 .. 256 */
    double dt;               /* step [s], > 0 */
    double lambda;           /* temperature of Eq. 4a, > 0 */
    double sigma[MPPI_NJ];   /* noise std per joint [N m], >= 0 (Eq. 2) */
    double W_pos[3], W_ori[3], W_force[6], W_reg[6];
    double w_q, w_qd, w_tau, w_post;
    double q_rest[MPPI_NJ];
    double w_terminal;
    int force_mode;          /* 0: tau_F = v - g(q) (default); 1: tau_F = v (Eq. 13) */
    int ext_mode;            /* mppi_ext_mode */
    double F_ext[6];         /* EXT_CONST: world wrench; tau_ext = J(q_0)^T F_ext held
                                over the horizon (Sec. III-A) */
    double wall_n[3];        /* EXT_WALL: unit normal, plane n.p = wall_d0; force
                                n * max(0, k delta + c d(delta)/dt), delta = d0 - n.p_ee */
    double wall_d0, wall_k, wall_c;
    int precision;           /* mppi_precision of the rollouts */
    double lambda_fp64_threshold; /* weights and weighted sum in FP64 when
                                     lambda < threshold (FP32 otherwise) */
    /* Collision term of Eqs. 14-15: C_collision = w_collision times the
     * number of pairs whose minimum segment distance d_i is below d_th[i],
     * added to the running cost at every pre-step state (not to phi).
     * Segment ids: 0..6 are the links (link i runs from the origin of
     * joint i to that of joint i+1, link 6 to the EE point; cylinder radii
     * go into the thresholds), 7 + o is obstacle o, a world segment held
     * over the horizon (change it between updates with mppi_set_cost). */
    double w_collision;      /* >= 0 */
    int n_obstacles;         /* 0 .. MPPI_MAX_OBSTACLES */
    double obstacles[MPPI_MAX_OBSTACLES][6];  /* end a [3], end b [3], world [m] */
    int n_pairs;             /* 0 .. MPPI_MAX_PAIRS; 0 disables the term */
    int pairs[MPPI_MAX_PAIRS][2];             /* segment ids, < 7 + n_obstacles */
    double d_th[MPPI_MAX_PAIRS];              /* thresholds [m], >= 0 */
    int dynamics;            /* mppi_dynamics (single-problem solvers; batches
                                and the nominal selection use MPPI_DYN_ABA) */
    /* Sampling variants (the paper defers its sampling strategy to a cited
     * work, end of Sec. III-B; these are two common choices).  noise_rho in [0, 1): the
     * perturbation of Eq. 2 becomes an AR(1) process in time,
     * du_0 = sigma z_0, du_t = rho du_{t-1} + sqrt(1 - rho^2) sigma z_t, with
     * the marginal variance sigma^2 at every step (0: independent draws).
     * iterations in 0 .. MPPI_MAX_ITERATIONS (0 and 1: one update): an update
     * runs that many MPPI iterations on the same state, each from the
     * previous one's U_new, iteration i drawing its noise with the Philox
     * tick word iterations * tick + i; costs, noise and status are the last
     * iteration's.  The problems of a batch must share one iteration count;
     * the stage-isolated calls (mppi_rollout_async, mppi_weights_async)
     * take one iteration only (MPPI_ENOTSUP otherwise). */
    double noise_rho;
    int iterations;
} mppi_cost_params;

typedef struct {
    double p_des[3];
    double quat_des[4];      /* w x y z, normalised on use */
    double F_des[6];         /* desired EE wrench [force; moment] */
} mppi_target;

typedef struct mppi_solver* mppi_handle_t;

/* Creates a solver.  Copies both structs (the caller may free them);
 * validates them; allocates device buffers for (K, T): noise K*T*7 and
 * costs K in the rollout precision, plus small staging buffers.
 * Errors: MPPI_EINVAL (null, n_joints != 7, K or T out of range, dt <= 0,
 * lambda <= 0, sigma < 0, mass <= 0, inertia not PD or violating the
 * triangle inequality, non-finite field, unknown mode), MPPI_ENOMEM,
 * MPPI_EDEVICE (no usable GPU). */
int mppi_create(const mppi_robot_params* robot, const mppi_cost_params* cost,
                mppi_handle_t* out);

/* Releases everything the handle owns.  NULL is accepted. */
int mppi_destroy(mppi_handle_t h);

/* Replaces the cost settings (same K and T as at create; MPPI_EINVAL
 * otherwise).  Takes effect for later updates. */
int mppi_set_cost(mppi_handle_t h, const mppi_cost_params* cost);

/* Launch shape of the updates: 2 runs each group of 64
 * samples on two waves where supported (FP32 rollouts of the
 * articulated-body route): one wave integrates the dynamics while the
 * other draws the next step's perturbations and evaluates the force
 * estimate (Eq. 13) and the cost of the previous step, which shortens the
 * per-step critical path; FP64 rollouts, the route of Eq. 8, and 1 use one
 * wave per 64 samples (the same arithmetic per sample as 2).  8 gives
 * every sample eight lanes of a wave, one per joint and one for the EE
 * frame (the default; FP32 rollouts of the articulated-body route,
 * elsewhere it acts as 2): kinematics, twists and bias
 * forces by scans over the lanes, the inertia of Eq. 8 from
 * composite-rigid-body inertias, Eq. 6 by an LDL^T solve, the force
 * estimate of Eq. 13 with its right-hand sides split over the lanes and
 * the collision pairs of Eq. 15 dealt over them; the
 * forward dynamics are the same quantity by another factorisation, so
 * results agree with the other shapes to FP32 rounding.
 * Errors: MPPI_EINVAL (null, other values). */
int mppi_set_launch(mppi_handle_t h, int waves_per_group);

/* Synchronous update from host memory (Sec. II: one MPPI iteration).
 *   q, qd      [7] measured state x_0
 *   target     pose / wrench targets
 *   U_nominal  [T][7] nominal torques u_t (row-major)
 *   seed, tick Philox key and the tick word of the counter
 *   U_new      [T][7] out; may alias U_nominal
 *   costs      [K] out, may be NULL: S_k as computed (rollout precision,
 *              widened), +inf for non-finite samples
 * Returns MPPI_ENONFINITE (with U_new = U_nominal) if no S_k is finite. */
int mppi_update(mppi_handle_t h, const double* q, const double* qd,
                const mppi_target* target, const double* U_nominal,
                uint64_t seed, uint64_t tick, double* U_new, double* costs);

/* Device-side I/O of one update.  All pointers are device memory.
 * The element type of costs and noise is that of the rollout precision
 * (float for MPPI_FP32, double for MPPI_FP64). */
typedef struct {
    const double* q;          /* [7] */
    const double* qd;         /* [7] */
    const double* target;     /* [13]: p_des[3], quat_des[4], F_des[6] */
    const double* U_nominal;  /* [T][7] */
    double* U_new;            /* [T][7] out (may alias U_nominal) */
    double* U_shift;          /* [T][7] out or NULL: U_new shifted one step,
                                 last row repeated (the warm start, Sec. II) */
    void* costs;              /* [K] out or NULL (then an internal buffer is used) */
    void* noise;              /* [T][7][K] out or NULL (internal buffer) */
    int* status;              /* [1] out or NULL: MPPI_OK / MPPI_ENONFINITE */
    uint64_t seed, tick;
} mppi_device_io;

/* Enqueues one update on `stream` (a hipStream_t; NULL = default stream):
 * the rollout kernel (noise, dynamics, cost, per-workgroup partials of
 * Eq. 4) and the merge of the partials, fused into the rollout launch for
 * the per-lane launch shapes and a second launch for the eight-lane one.
 * The caller synchronises.  Errors: MPPI_EINVAL, MPPI_EDEVICE. */
int mppi_update_async(mppi_handle_t h, const mppi_device_io* io, void* stream);

/* Picks the launch shape of mppi_set_launch (8, 2 or 1) by timing updates
 * of this problem on `stream` with the caller's io (device pointers as for
 * mppi_update_async; its outputs are written by the timing runs; a
 * representative state gives representative times): per shape one untimed
 * update, then about budget_ms / 3 of timed ones.  Sets the handle's shape,
 * returns it in *best_launch (may be NULL) and the mean update times in
 * times_ms[3] (launch 8, 2, 1; may be NULL).  With an autotune cache the
 * choice is stored under (architecture, K, T, precision, dynamics route,
 * cost terms, iterations) and reused without timing (times_ms set to -1).
 * Errors: MPPI_EINVAL (null, budget_ms < 1), MPPI_EDEVICE. */
int mppi_autotune(mppi_handle_t h, const mppi_device_io* io, int budget_ms, void* stream,
                  int* best_launch, float* times_ms);

/* Autotune cache of mppi_autotune and mppi_batch_autotune: a JSON file at
 * `path` (one object, one entry per key: the chosen shape and its time),
 * read when a tuner starts and rewritten (via a temporary file and a
 * rename) when it stores a new choice.  NULL or "" turns the cache off (the
 * default).  Process-wide; the string is copied. */
int mppi_set_autotune_cache(const char* path);

/* The update of mppi_update_async without allocating anything, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  No handle: robot
 * and cost are validated as mppi_create validates them (host structs, read
 * during the call only), and io is as for mppi_update_async (device
 * pointers in the element type of cost->precision; io->costs and io->noise
 * may be NULL).  Runs the default launch shape.  What the update needs
 * beyond io lives in a static device workspace of 8 MiB per GPU (held
 * until the process ends): the prepared model and cost, written by a
 * set-up kernel whose arguments carry them by value, a cleared counter,
 * the intermediate sequences of several iterations (34 KB in all), the
 * Eq. 4 partials (ceil(K / 16) (2 + 7 T) doubles) and, when io->costs is
 * NULL, the costs (K values).  Enqueues the set-up kernel and the update
 * on `stream`; the caller synchronises.  Every call on a GPU uses that
 * GPU's one workspace, so calls that overlap in time on one GPU race
 * (serialise them, e.g. on one stream).
 * Errors: MPPI_EINVAL (as mppi_create and mppi_update_async),
 * MPPI_ESCRATCH (the sizes above exceed 8 MiB, e.g. K > 32768 at T = 64;
 * nothing is launched), MPPI_EDEVICE. */
int mppi_update_noalloc(const mppi_robot_params* robot, const mppi_cost_params* cost,
                        const mppi_device_io* io, void* stream);

/* Stage entry points (the two halves of mppi_update_async, same io):
 * rollout only writes costs and noise; weights reads them (Eq. 4) and
 * writes U_new, U_shift and status. */
int mppi_rollout_async(mppi_handle_t h, const mppi_device_io* io, void* stream);
int mppi_weights_async(mppi_handle_t h, const mppi_device_io* io, void* stream);

/* Closed-loop plant on the device (the zero-order hold of the paper's
 * experimental setup): holds torque u (clamped to tau_max) for `dt`
 * seconds in `substeps` semi-implicit Euler substeps of FP64 forward
 * dynamics with the handle's external-wrench model.  q, qd [7] device,
 * updated in place; u [7] device. */
int mppi_plant_step_async(mppi_handle_t h, double* q, double* qd,
                          const double* u, double dt, int substeps,
                          void* stream);

/* mppi_plant_step_async with a further world wrench [force; moment] (N,
 * N m) acting at the EE point, e.g. a push on the end effector that the
 * controller does not model (the external perturbations of the free-space
 * experiment, Sec. IV-B): J(q)^T wrench is added to the clamped torque at
 * every substep, at that substep's state.  wrench: device [6], or NULL
 * (then exactly mppi_plant_step_async).  Errors as mppi_plant_step_async. */
int mppi_plant_step_wrench_async(mppi_handle_t h, double* q, double* qd,
                                 const double* u, const double* wrench,
                                 double dt, int substeps, void* stream);

/* EE pose of n states of the handle's arm, FP64 forward kinematics (the
 * EE frame of Sec. III-A, Fig. 1 caption): q device [n][7]; pose device
 * [n][7] = position [3] (m, world) then the unit quaternion (w, x, y, z)
 * of the EE frame with w >= 0.  Enqueued on `stream`.  Errors: MPPI_EINVAL
 * (null pointer, n < 1), MPPI_EDEVICE. */
int mppi_ee_pose_async(mppi_handle_t h, const double* q, int n, double* pose,
                       void* stream);

/* ---- batched problems (one persistent launch per control tick) ---- */

typedef struct mppi_batch* mppi_batch_t;

/* One problem of a batch: its own arm and cost (K, T, weights, lambda).
 * Rollouts run in FP32 (cost->precision must be MPPI_FP32) and T must be
 * at most 64. */
typedef struct {
    const mppi_robot_params* robot;
    const mppi_cost_params* cost;
} mppi_problem_desc;

/* Creates a batch of n >= 1 problems.  Copies every struct; validates each
 * problem as mppi_create does; builds the work list (64-sample tiles,
 * longest horizon first) and the device tables.  Errors: MPPI_EINVAL,
 * MPPI_ENOTSUP (FP64, T > 64, the explicit-M dynamics or iteration counts
 * that differ between problems), MPPI_ENOMEM, MPPI_EDEVICE. */
int mppi_batch_create(const mppi_problem_desc* descs, int n, mppi_batch_t* out);
int mppi_batch_destroy(mppi_batch_t b);

/* Layout of the packed arrays: problem p's U rows start at u_off[p]
 * (in doubles, [T_p][7]) and its costs at k_off[p] (in floats).  Either
 * output array may be NULL; totals are written when the pointers are
 * non-NULL. */
int mppi_batch_layout(mppi_batch_t b, size_t* u_off, size_t* k_off, size_t* u_total, size_t* k_total);

/* Device I/O of a batched update.  All pointers are device memory. */
typedef struct {
    const double* q;          /* [n][7] */
    const double* qd;         /* [n][7] */
    const double* target;     /* [n][13]: p_des, quat_des, F_des */
    const double* U_nominal;  /* packed [sum T][7] */
    double* U_new;            /* packed [sum T][7] out (may alias U_nominal) */
    double* U_shift;          /* packed [sum T][7] out or NULL (must not alias the others) */
    float* costs;             /* packed [sum K] out or NULL */
    int* status;              /* [n] out or NULL */
    const uint64_t* seed;     /* [n] Philox keys */
} mppi_batch_io;

/* Enqueues one batched update with Philox tick `tick` on `stream`. */
int mppi_batch_update_async(mppi_batch_t b, const mppi_batch_io* io, uint64_t tick, void* stream);

/* Launch shape: waves per workgroup and workgroup count.  1, 2 or 4: one
 * lane per sample, every wave takes 64-sample tiles from the work list (the
 * articulated-body rollouts); 8: eight lanes per sample, a workgroup of
 * eight waves takes a 64-sample tile together (eight samples per wave, the
 * eight-lane arithmetic of mppi_set_launch(h, 8) with each step's dynamics
 * and cost on one wave).  Both write the same partials of Eq. 4, so they
 * give the same U_new to FP32 rounding. */
int mppi_batch_set_launch(mppi_batch_t b, int waves_per_group, int groups);

/* Times every launch shape of the built-in search space (waves per
 * workgroup {1, 2, 4, 8}, i.e. one lane per sample in workgroups of 1, 2 or
 * 4 waves, or eight lanes per sample, x resident waves {256, 512, 1024,
 * 2048}) with `reps` updates each on `stream`, keeps the fastest and
 * returns it.  times_ms (may be NULL) receives the 16 mean times in search
 * order.  The io buffers are written by the timing runs.  With an autotune
 * cache (mppi_set_autotune_cache) the choice is stored under a key of the
 * device architecture, the batch's total sample-steps (power-of-two
 * bucket), its horizon range, the precision, the union of its cost terms
 * and the iteration count; a later call with the same key takes the stored
 * shape without timing and sets every times_ms entry to -1. */
int mppi_batch_autotune(mppi_batch_t b, const mppi_batch_io* io, int reps, void* stream,
                        int* best_waves_per_group, int* best_groups, float* times_ms);

/* Captures one batched update with these io pointers (which must stay
 * valid) into a HIP graph: the update reads the Philox tick from a device
 * slot of the graph and then advances it by one.  mppi_batch_set_tick sets
 * that slot (synchronous; eager mppi_batch_update_async calls use a slot of
 * their own and never move it); mppi_batch_graph_launch replays the graph
 * on `stream`.  Replays and eager calls share the batch's work queue, so
 * they must not overlap in time. */
int mppi_batch_graph_capture(mppi_batch_t b, const mppi_batch_io* io);
int mppi_batch_set_tick(mppi_batch_t b, uint64_t tick);
int mppi_batch_graph_launch(mppi_batch_t b, void* stream);

/* Advances every problem's measured state (io->q, io->qd, written in place;
 * the io struct's const is cast away for these two) by dt seconds of the
 * FP64 zero-order-hold plant of mppi_plant_step_async, holding the first
 * row of the problem's io->U_new (clamped to the torque limits).  One
 * workgroup per problem. */
int mppi_batch_plant_step_async(mppi_batch_t b, const mppi_batch_io* io, double dt, int substeps, void* stream);

/* ---- warm start for a solver period that differs from dt ---- */

/* Receding horizon (Sec. II: the rest of the optimised sequence seeds the
 * next update) after shift_steps = s horizon steps of elapsed time (the
 * solver period over dt): U_new is read as piecewise constant in time (row
 * t held over [t dt, (t+1) dt), the last row held past the horizon) and row
 * t of U_out is its mean over [(t + s) dt, (t + s + 1) dt), i.e.
 *   (1 - f) U_new[min(t + m, T-1)] + f U_new[min(t + m + 1, T-1)],
 * m = floor(s), f = s - m.  s = 1 gives U_shift of an update bit for bit.
 * Device [T][7] buffers that must not overlap; 0 <= s <= T.
 * Errors: MPPI_EINVAL (null, overlap, s out of range or non-finite),
 * MPPI_EDEVICE. */
int mppi_warm_start_async(mppi_handle_t h, const double* U_new, double* U_out, double shift_steps, void* stream);
/* The same for every problem of a batch, in the packed layout
 * (0 <= s <= 64). */
int mppi_batch_warm_start_async(mppi_batch_t b, const double* U_new, double* U_out, double shift_steps,
                                void* stream);

/* ---- nominal-sequence selection (plain MPPI as the fallback) ---- */

/* Rolls out two sequences from the state of `io` without noise (the same
 * dynamics and cost as an update, sigma taken as 0): io->U_nominal (the
 * plain warm start, candidate 0) and U_candidate ([T][7], device,
 * candidate 1), and replaces the content of io->U_nominal (written through
 * the pointer: it must be writable device memory) with U_candidate only
 * when its cost is lower (a tie keeps the warm start).  costs (device
 * double [2] or NULL) receives both costs.  Errors: MPPI_EINVAL. */
int mppi_select_nominal_async(mppi_handle_t h, const mppi_device_io* io, const double* U_candidate, double* costs,
                              void* stream);
/* The same for every problem of a batch, one workgroup each; U_candidates
 * in the packed layout of U_nominal, costs (device double [n][2] or NULL). */
int mppi_batch_select_nominal_async(mppi_batch_t b, const mppi_batch_io* io, const double* U_candidates,
                                    double* costs, void* stream);

/* ---- learned proposal network ----
 *
 * An addition to the method, whose sampling of Eq. 2 centres on the shifted
 * warm start: a multilayer perceptron maps the measured state and the pose
 * target to a mean torque sequence over an 18-step horizon, which the
 * selection above offers to plain MPPI as an alternative nominal sequence.
 *
 *   x = (q / q_max, qd / qd_max, p_des, quat_des) in R^21 (quaternion
 *       normalised, sign chosen so that w >= 0; limits from the robot)
 *   z_l = W_l a_{l-1} + b_l, a_l = gelu(z_l) for l = 1, 2, 3 (tanh form of
 *       GELU), widths 21-256-256-256-126; y = W_4 a_3 + b_4
 *   U[t][j] = tau_max_j y[7 t + j]
 *   training loss L = sum (y - y*)^2 / (B 126), y* = U* / tau_max
 *
 * BF16 weights, input features, hidden activations and backward signals
 * (round to nearest even) with FP32 accumulation on the matrix cores; FP32
 * biases; FP32 master weights and moments for Adam.  Parameters are passed
 * flat in the order W_1 [256][21], b_1, W_2 [256][256], b_2, W_3, b_3,
 * W_4 [126][256], b_4 (row-major [out][in]); MPPI_MLP_PARAMS values. */
#define MPPI_MLP_INPUTS 21
#define MPPI_MLP_OUTPUTS 126
#define MPPI_MLP_PARAMS 169598

typedef struct mppi_mlp* mppi_mlp_t;

typedef struct {
    double lr, beta1, beta2, eps;   /* Adam (Kingma and Ba), bias-corrected */
} mppi_adam_params;

/* Creates a network for `robot` (feature and torque scales) with room for
 * batches of up to max_batch rows (1 .. 65536).  Parameters start at zero;
 * set them before use.  Errors: MPPI_EINVAL, MPPI_ENOMEM, MPPI_EDEVICE. */
int mppi_mlp_create(const mppi_robot_params* robot, int max_batch, mppi_mlp_t* out);
int mppi_mlp_destroy(mppi_mlp_t m);
/* Host FP32 parameters in and out (n must be MPPI_MLP_PARAMS; synchronous).
 * Setting them also clears the Adam moments and step count. */
int mppi_mlp_set_params(mppi_mlp_t m, const float* params, size_t n);
int mppi_mlp_get_params(mppi_mlp_t m, float* params, size_t n);
/* y [B][126] = network(x [B][21]) (device FP32, 1 <= B <= max_batch). */
int mppi_mlp_forward_async(mppi_mlp_t m, const float* x, int B, float* y, void* stream);
/* Loss and gradient of one batch (x [B][21], y_target [B][126]): the
 * gradient stays in the network for mppi_mlp_adam_async and is copied to
 * grad (device FP32 [MPPI_MLP_PARAMS] in the flat order) when non-NULL;
 * loss (device FP32 [1]) may be NULL. */
int mppi_mlp_grad_async(mppi_mlp_t m, const float* x, const float* y_target, int B, float* grad, float* loss,
                        void* stream);
/* One Adam step with the last gradient (the step count t advances on the
 * host with every call). */
int mppi_mlp_adam_async(mppi_mlp_t m, const mppi_adam_params* p, void* stream);
/* The same result as mppi_mlp_grad_async (no gradient copy) followed by
 * mppi_mlp_adam_async, in two kernel launches: the Adam step of each
 * parameter is applied as its gradient tile completes. */
int mppi_mlp_train_step_async(mppi_mlp_t m, const float* x, const float* y_target, int B,
                              const mppi_adam_params* p, float* loss, void* stream);
/* Mean torque sequences of n states (1 <= n <= max_batch): q, qd [n][7],
 * target [n][13] (the update's layout; F_des unused) in, U [n][u_stride]
 * doubles out (the first 126 of each row: [18][7]); all device memory.
 * One kernel launch: the input features are encoded in its input load. */
int mppi_mlp_propose_async(mppi_mlp_t m, int n, const double* q, const double* qd, const double* target,
                           double* U, int u_stride, void* stream);

/* Training rows from n recorded (state, target, solution) triples: x
 * [n][21] features (as the proposal computes them) and, when y is non-NULL,
 * y [n][126] = U [n][u_stride] / tau_max (U [t][j] row-major in the first
 * 126 values of each row).  Device memory; n is not bounded by max_batch. */
int mppi_mlp_encode_async(mppi_mlp_t m, int n, const double* q, const double* qd, const double* target,
                          const double* U, int u_stride, float* x, float* y, void* stream);

/* Human-readable name of a status code (static storage). */
const char* mppi_strerror(int status);

/* Build/version string (static storage). */
const char* mppi_version(void);

#ifdef __cplusplus
}
#endif
#endif
