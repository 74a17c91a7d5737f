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
 *   - each rolled out for T steps through 7-DoF forward dynamics (Eqs. 5-6,
 *     computed with the articulated-body algorithm) and the semi-implicit
 *     Euler step written in Eq. 7;
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

typedef enum {
    MPPI_OK = 0,
    MPPI_EINVAL = 1,      /* bad argument (null, size, non-finite, range) */
    MPPI_ENONFINITE = 2,  /* every sample cost was non-finite: U_new = U_nominal */
    MPPI_ENOMEM = 3,      /* device or pinned host allocation failed */
    MPPI_EDEVICE = 4,     /* a HIP runtime call or kernel launch failed */
    MPPI_ENOTSUP = 5      /* valid request this build does not implement */
} mppi_status;

typedef enum { MPPI_FP32 = 0, MPPI_FP64 = 1 } mppi_precision;
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
 * the rollout kernel (noise, dynamics, cost) then the weighting kernel.
 * The caller synchronises.  Errors: MPPI_EINVAL, MPPI_EDEVICE. */
int mppi_update_async(mppi_handle_t h, const mppi_device_io* io, void* stream);

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
 * MPPI_ENOTSUP (FP64 or T > 64), MPPI_ENOMEM, MPPI_EDEVICE. */
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

/* Launch shape: waves per workgroup (1, 2 or 4) and workgroup count. */
int mppi_batch_set_launch(mppi_batch_t b, int waves_per_group, int groups);

/* Times every launch shape of the built-in search space (waves per
 * workgroup {1, 2, 4} x resident waves {256, 512, 1024, 2048}) with `reps`
 * updates each on `stream`, keeps the fastest and returns it.  times_ms
 * (may be NULL) receives the 12 mean times in search order.  The io buffers
 * are written by the timing runs. */
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

/* Human-readable name of a status code (static storage). */
const char* mppi_strerror(int status);

/* Build/version string (static storage). */
const char* mppi_version(void);

#ifdef __cplusplus
}
#endif
#endif
