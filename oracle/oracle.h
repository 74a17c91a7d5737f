/*
 * oracle.h -- plain, slow, FP64 CPU oracle for torque-sampling MPPI with
 * analytic rigid-body dynamics (Im et al., "Real-Time Dynamics-Based
 * Torque-Sampling MPPI for Compliant and Force Aware Manipulation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes this
 * header, links this code or calls it.  It exists so that tests, the smoke
 * check and the CPU baseline leg of the benchmark can compare the HIP path
 * against an independent, obviously-correct implementation written from the
 * paper.  It shares no code, header or constant with the HIP path.
 *
 * Conventions (all FP64, row-major):
 *   - Serial chain of n <= ORA_MAXJ revolute joints; joint i rotates about
 *     the z axis of its own frame.  Frame i relative to frame i-1:
 *     orientation R_parent_i * Rz(q_i), origin r_parent_i (in frame i-1).
 *   - Frame 0 is the world; gravity is a world vector (default 0,0,-9.81).
 *   - Link inertia is about the link CoM, expressed in link-frame axes.
 *   - Task-space vectors are world-aligned; wrenches/twists are ordered
 *     [linear; angular] as in the paper's Jacobian J = [J_v; J_w].
 */
#ifndef MPPI_ORACLE_H
#define MPPI_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORA_MAXJ 7
#define ORA_MAXOBS 4
#define ORA_MAXPAIRS 32

typedef struct {
    double R_parent[9];  /* rotation of joint frame i in frame i-1 (before Rz(q_i)) */
    double r_parent[3];  /* origin of frame i in frame i-1 coordinates [m] */
    double mass;         /* [kg] */
    double com[3];       /* CoM in frame i [m] */
    double inertia[6];   /* about CoM, frame-i axes: xx yy zz xy xz yz [kg m^2] */
    double armature;     /* rotor inertia added on the joint diagonal [kg m^2] */
    double q_min, q_max; /* joint position limits [rad] */
    double qd_max;       /* joint speed limit [rad/s] */
    double tau_max;      /* torque limit [N m] */
} ora_link;

typedef struct {
    int n;                    /* number of joints, 1..ORA_MAXJ */
    ora_link link[ORA_MAXJ];
    double R_ee[9];           /* end-effector frame in the last link frame */
    double r_ee[3];           /* end-effector point in the last link frame */
    double gravity[3];        /* world gravity vector [m/s^2] */
} ora_robot;

enum { ORA_EXT_NONE = 0, ORA_EXT_CONST = 1, ORA_EXT_WALL = 2 };

typedef struct {
    int K, T;                 /* samples, horizon steps */
    double dt;                /* step [s] */
    double lambda;            /* temperature */
    double sigma[ORA_MAXJ];   /* noise std per joint [N m] */
    double W_pos[3], W_ori[3], W_force[6], W_reg[6];
    double w_q, w_qd, w_tau, w_post;
    double q_rest[ORA_MAXJ];
    double w_terminal;
    int force_mode;           /* 0: tau_F = v - g(q); 1: tau_F = v */
    int ext_mode;             /* ORA_EXT_* */
    double F_ext[6];          /* constant external wrench [force; moment], world */
    double wall_n[3];         /* unit wall normal (points out of the wall) */
    double wall_d0;           /* wall plane: n . p = d0 */
    double wall_k, wall_c;    /* spring [N/m], damper [N s/m] */
    /* collision term of Eqs. (14)-(15): w_collision * #{pairs with d < d_th};
       segment ids 0..n-1 are the links (link i from the origin of joint i to
       that of joint i+1, the last one to the EE point), n + o is obstacle o */
    double w_collision;
    int n_obstacles;                       /* 0..ORA_MAXOBS */
    double obstacles[ORA_MAXOBS][6];       /* world segments: end a, end b [m] */
    int n_pairs;                           /* 0..ORA_MAXPAIRS */
    int pairs[ORA_MAXPAIRS][2];            /* segment ids */
    double d_th[ORA_MAXPAIRS];             /* thresholds [m] */
    /* sampling variants: du_t = rho du_{t-1} + sqrt(1 - rho^2) sigma z_t
       (du_0 = sigma z_0; rho = 0 is the i.i.d. noise of Eq. 2), and
       `iterations` MPPI updates per call, each from the previous U_new,
       iteration i using the Philox tick iterations * tick + i */
    double noise_rho;                      /* 0 <= rho < 1 */
    int iterations;                        /* <= 1: one update */
} ora_cost;

typedef struct {
    double p_des[3];
    double quat_des[4];       /* w, x, y, z (normalised on use) */
    double F_des[6];          /* desired EE wrench [force; moment], world */
} ora_target;

enum { ORA_OK = 0, ORA_EINVAL = 1, ORA_ENONFINITE = 2, ORA_ESINGULAR = 3 };

/* ---- kinematics ---------------------------------------------------- */
/* World frames of all links plus the EE: R[i*9], p[i*3] for i < n. */
void ora_fk(const ora_robot* rb, const double* q, double* R, double* p,
            double* p_ee, double* R_ee);
/* EE Jacobian, 6 x n row-major, rows [J_v; J_w], world-aligned, at p_ee. */
void ora_ee_jacobian(const ora_robot* rb, const double* q, double* J);

/* ---- dynamics ------------------------------------------------------ */
/* Mass matrix by the paper's Jacobian sum (Eq. 8), n x n row-major. */
void ora_mass_jacobian_sum(const ora_robot* rb, const double* q, double* M);
/* Bias h(q, qd) from link Jacobians and their time derivatives. */
void ora_bias_jacobian(const ora_robot* rb, const double* q, const double* qd,
                       double* h);
/* Spatial-algebra pins: composite-rigid-body M, recursive Newton-Euler
   inverse dynamics (with armature), articulated-body forward dynamics.
   f_ee: optional world wrench [force; moment] applied at the EE point. */
void ora_crba(const ora_robot* rb, const double* q, double* M);
void ora_rnea(const ora_robot* rb, const double* q, const double* qd,
              const double* qdd, const double* f_ee, double* tau);
void ora_aba(const ora_robot* rb, const double* q, const double* qd,
             const double* tau, const double* f_ee, double* qdd);
/* qdd = M^{-1}(tau + J^T f_ee - h) using Eq. 8 M, Jacobian h, Cholesky. */
int  ora_forward_dynamics(const ora_robot* rb, const double* q,
                          const double* qd, const double* tau,
                          const double* f_ee, double* qdd);
/* Dense Cholesky solve of an SPD system (A is n x n, b overwritten). */
int  ora_cholesky_solve(int n, const double* A, double* b);
/* Kinetic + potential energy (armature included in the kinetic part). */
double ora_energy(const ora_robot* rb, const double* q, const double* qd);

/* ---- task space ----------------------------------------------------- */
void ora_quat_to_R(const double* quat, double* R);
/* Rotation vector of a rotation matrix (the SO(3) log map). */
void ora_so3_log(const double* R, double* rho);
/* F_ee = Jbar^T tau_F, Jbar = M^-1 J^T (J M^-1 J^T)^-1 (Eq. 13). */
int  ora_force_estimate(const ora_robot* rb, const double* q,
                        const double* tau_F, double* F_ee);
/* Wall contact wrench at the EE (force only) for the wall model. */
void ora_wall_force(const ora_cost* c, const double* p_ee,
                    const double* v_ee, double* F);

/* ---- noise ---------------------------------------------------------- */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4]);
/* 8 standard normals for (seed, tick, sample k, step t). */
void ora_normals(uint64_t seed, uint64_t tick, uint32_t k, uint32_t t,
                 double z[8]);

/* ---- costs ---------------------------------------------------------- */
/* Running cost l(x_t, v_t) (Eqs. 9-14) and terminal cost phi(x_T).
   parts (optional, 6): pos, ori, force, joint, torque, total. */
double ora_running_cost(const ora_robot* rb, const ora_cost* c,
                        const ora_target* tg, const double* q,
                        const double* qd, const double* v, double* parts);
/* Minimum distance between the segments [a0, a1] and [b0, b1]. */
double ora_segment_distance(const double* a0, const double* a1, const double* b0, const double* b1);
/* The n link segments at q: seg[i*6 .. i*6+5] = (start, end). */
void ora_link_segments(const ora_robot* rb, const double* q, double* seg);
/* C_collision of Eq. (15) at q; *margin (may be NULL) receives
   min_i |d_i - d_th,i| (infinity without pairs). */
double ora_collision_cost(const ora_robot* rb, const ora_cost* c, const double* q, double* margin);
double ora_terminal_cost(const ora_robot* rb, const ora_cost* c,
                         const ora_target* tg, const double* q,
                         const double* qd);

/* ---- MPPI ----------------------------------------------------------- */
/* Roll out one sample; returns S_k.  noise (optional): T x n. */
double ora_rollout(const ora_robot* rb, const ora_cost* c,
                   const ora_target* tg, const double* q0, const double* qd0,
                   const double* U_nom, uint64_t seed, uint64_t tick,
                   uint32_t k, double* noise);
/* The same rollout; also returns, in *margin, the smallest |d_i - d_th,i|
   over every pre-step state of the horizon (the collision indicator's
   distance to a flip). */
double ora_rollout_margin(const ora_robot* rb, const ora_cost* c,
                          const ora_target* tg, const double* q0, const double* qd0,
                          const double* U_nom, uint64_t seed, uint64_t tick,
                          uint32_t k, double* noise, double* margin);
/* Eq. 4 weighting of given costs and noise (K x T x n) into U_new. */
int  ora_weights_update(int K, int T, int n, double lambda, const double* S,
                        const double* noise, const double* U_nom,
                        double* U_new, double* weights);
/* One full MPPI update.  costs (K) and noise (K x T x n) optional.
   nthreads <= 0: use the OpenMP default. */
int  ora_update(const ora_robot* rb, const ora_cost* c, const ora_target* tg,
                const double* q0, const double* qd0, const double* U_nom,
                uint64_t seed, uint64_t tick, double* U_new, double* costs,
                double* noise, int nthreads);
/* Receding-horizon warm start after s >= 0 horizon steps of elapsed time
   (Sec. II: the rest of the optimised sequence seeds the next update).  The
   sequence U (T x n) is read as piecewise constant in time, row i held over
   [i, i+1) in units of dt and the last row held past the horizon; row t of
   out is its mean over [t + s, t + s + 1).  s = 1 is the one-step shift. */
void ora_warm_start(int T, int n, const double* U, double s, double* out);
/* Closed-loop plant: hold torque u (clamped to tau_max) for dt using
   `substeps` semi-implicit Euler substeps with the wall/constant wrench. */
void ora_plant_step(const ora_robot* rb, const ora_cost* c, double* q,
                    double* qd, const double* u, double dt, int substeps);
/* Threads the OpenMP runtime will use. */
int  ora_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
