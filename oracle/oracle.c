/*
 * oracle.c -- FP64 CPU oracle for torque-sampling MPPI (TEST INFRASTRUCTURE).
 *
 * Written from the paper (Im et al., "Real-Time Dynamics-Based Torque-
 * Sampling MPPI for Compliant and Force Aware Manipulation"), section
 * numbers and equation numbers as printed there:
 *   Sec. II    Eqs. (1)-(4): stochastic system, perturbed control, OCP cost,
 *              importance weights with the minimum-cost shift.
 *   Sec. III-A Eqs. (5)-(8): rigid-body dynamics, forward dynamics solve,
 *              Euler integration, Jacobian-sum mass matrix; bias h from the
 *              link Jacobians and their time derivatives.
 *   Sec. III-B Eqs. (9)-(14): running cost, motion/force/constraint terms,
 *              dynamically consistent force estimate.
 *
 * The rollout follows the paper's own route (FK -> link Jacobians and their
 * derivatives -> M by Eq. 8, h -> Cholesky solve of Eq. 6 -> Eq. 7).  The
 * spatial-algebra algorithms (CRBA, RNEA, ABA) are here only as pins for
 * the dynamics; the HIP path uses its own articulated-body code and shares
 * nothing with this file.  Where the paper is silent the reading used is
 * stated at the function.
 *
 * Only tests, the smoke check and the benchmark's CPU-baseline leg call this.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define N ORA_MAXJ

/* ------------------------------------------------------------------ */
/* small dense helpers (3-vectors, 3x3 row-major, 6x6 row-major)      */
/* ------------------------------------------------------------------ */
static void v3_cross(const double* a, const double* b, double* c)
{
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    c[0] = x; c[1] = y; c[2] = z;
}
static double v3_dot(const double* a, const double* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void m3_mul(const double* A, const double* B, double* C)
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += A[i * 3 + k] * B[k * 3 + j];
            T[i * 3 + j] = s;
        }
    memcpy(C, T, sizeof T);
}
static void m3_vec(const double* A, const double* x, double* y)
{
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[i * 3] * x[0] + A[i * 3 + 1] * x[1] + A[i * 3 + 2] * x[2];
    y[0] = t[0]; y[1] = t[1]; y[2] = t[2];
}
static void m3_tvec(const double* A, const double* x, double* y)
{
    double t[3];
    for (int i = 0; i < 3; ++i) t[i] = A[i] * x[0] + A[3 + i] * x[1] + A[6 + i] * x[2];
    y[0] = t[0]; y[1] = t[1]; y[2] = t[2];
}
static void m3_transpose(const double* A, double* B)
{
    double T[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[j * 3 + i] = A[i * 3 + j];
    memcpy(B, T, sizeof T);
}
static void rotz(double q, double* R)
{
    double c = cos(q), s = sin(q);
    R[0] = c; R[1] = -s; R[2] = 0;
    R[3] = s; R[4] = c;  R[5] = 0;
    R[6] = 0; R[7] = 0;  R[8] = 1;
}
/* symmetric 3x3 from xx yy zz xy xz yz */
static void sym3(const double* s6, double* I)
{
    I[0] = s6[0]; I[4] = s6[1]; I[8] = s6[2];
    I[1] = I[3] = s6[3];
    I[2] = I[6] = s6[4];
    I[5] = I[7] = s6[5];
}
static void skew(const double* v, double* S)
{
    S[0] = 0;     S[1] = -v[2]; S[2] = v[1];
    S[3] = v[2];  S[4] = 0;     S[5] = -v[0];
    S[6] = -v[1]; S[7] = v[0];  S[8] = 0;
}
static void m6_zero(double* A) { memset(A, 0, 36 * sizeof(double)); }
static void m6_mul(const double* A, const double* B, double* C)
{
    double T[36];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0;
            for (int k = 0; k < 6; ++k) s += A[i * 6 + k] * B[k * 6 + j];
            T[i * 6 + j] = s;
        }
    memcpy(C, T, sizeof T);
}
static void m6_tmul(const double* A, const double* B, double* C) /* A^T B */
{
    double T[36];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) {
            double s = 0;
            for (int k = 0; k < 6; ++k) s += A[k * 6 + i] * B[k * 6 + j];
            T[i * 6 + j] = s;
        }
    memcpy(C, T, sizeof T);
}
static void m6_vec(const double* A, const double* x, double* y)
{
    double t[6];
    for (int i = 0; i < 6; ++i) {
        double s = 0;
        for (int k = 0; k < 6; ++k) s += A[i * 6 + k] * x[k];
        t[i] = s;
    }
    memcpy(y, t, sizeof t);
}
static void m6_tvec(const double* A, const double* x, double* y) /* A^T x */
{
    double t[6];
    for (int i = 0; i < 6; ++i) {
        double s = 0;
        for (int k = 0; k < 6; ++k) s += A[k * 6 + i] * x[k];
        t[i] = s;
    }
    memcpy(y, t, sizeof t);
}

/* ------------------------------------------------------------------ */
/* kinematics (Sec. III-A, Fig. 1 caption: joint transforms and CoM   */
/* offsets per link; each rollout computes EE pose and Jacobian)      */
/* ------------------------------------------------------------------ */
void ora_fk(const ora_robot* rb, const double* q, double* R, double* p,
            double* p_ee, double* R_ee)
{
    double Rprev[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double pprev[3] = {0, 0, 0};
    for (int i = 0; i < rb->n; ++i) {
        const ora_link* L = &rb->link[i];
        double Rz[9], Q[9], d[3];
        rotz(q[i], Rz);
        m3_mul(L->R_parent, Rz, Q);
        m3_vec(Rprev, L->r_parent, d);
        for (int a = 0; a < 3; ++a) p[i * 3 + a] = pprev[a] + d[a];
        m3_mul(Rprev, Q, &R[i * 9]);
        memcpy(Rprev, &R[i * 9], sizeof Rprev);
        memcpy(pprev, &p[i * 3], sizeof pprev);
    }
    if (p_ee) {
        double d[3];
        m3_vec(Rprev, rb->r_ee, d);
        for (int a = 0; a < 3; ++a) p_ee[a] = pprev[a] + d[a];
    }
    if (R_ee) m3_mul(Rprev, rb->R_ee, R_ee);
}

/* world axis of joint j: third column of R_j (Rz(q) keeps the z axis) */
static void axis_of(const double* R, int j, double* z)
{
    z[0] = R[j * 9 + 2]; z[1] = R[j * 9 + 5]; z[2] = R[j * 9 + 8];
}

/* Jacobian of a point x rigidly attached to link `upto` (columns > upto
   are zero): J_v col j = z_j x (x - p_j), J_w col j = z_j.  3 x n each. */
static void point_jacobian(int n, const double* R, const double* p, int upto,
                           const double* x, double* Jv, double* Jw)
{
    for (int j = 0; j < n; ++j) {
        double z[3], d[3], c[3];
        if (j > upto) {
            for (int a = 0; a < 3; ++a) { Jv[a * n + j] = 0; if (Jw) Jw[a * n + j] = 0; }
            continue;
        }
        axis_of(R, j, z);
        for (int a = 0; a < 3; ++a) d[a] = x[a] - p[j * 3 + a];
        v3_cross(z, d, c);
        for (int a = 0; a < 3; ++a) { Jv[a * n + j] = c[a]; if (Jw) Jw[a * n + j] = z[a]; }
    }
}

void ora_ee_jacobian(const ora_robot* rb, const double* q, double* J)
{
    int n = rb->n;
    double R[N * 9], p[N * 3], pe[3];
    double Jv[3 * N], Jw[3 * N];
    ora_fk(rb, q, R, p, pe, NULL);
    point_jacobian(n, R, p, n - 1, pe, Jv, Jw);
    for (int a = 0; a < 3; ++a)
        for (int j = 0; j < n; ++j) {
            J[a * n + j] = Jv[a * n + j];
            J[(3 + a) * n + j] = Jw[a * n + j];
        }
}

/* world CoM of each link and world inertia R_i I_i R_i^T */
static void link_world_inertial(const ora_robot* rb, const double* R,
                                const double* p, double* c, double* Iw)
{
    for (int i = 0; i < rb->n; ++i) {
        const ora_link* L = &rb->link[i];
        double d[3], I[9], T[9], Rt[9];
        m3_vec(&R[i * 9], L->com, d);
        for (int a = 0; a < 3; ++a) c[i * 3 + a] = p[i * 3 + a] + d[a];
        sym3(L->inertia, I);
        m3_mul(&R[i * 9], I, T);
        m3_transpose(&R[i * 9], Rt);
        m3_mul(T, Rt, &Iw[i * 9]);
    }
}

/* ------------------------------------------------------------------ */
/* Eq. (8): M = sum_i (J_r,i^T Ibar_i J_r,i + m_i J_c,i^T J_c,i)      */
/*              + diag(a),  Ibar_i = R_i I_i R_i^T                    */
/* ------------------------------------------------------------------ */
void ora_mass_jacobian_sum(const ora_robot* rb, const double* q, double* M)
{
    int n = rb->n;
    double R[N * 9], p[N * 3], c[N * 3], Iw[N * 9];
    ora_fk(rb, q, R, p, NULL, NULL);
    link_world_inertial(rb, R, p, c, Iw);
    memset(M, 0, sizeof(double) * n * n);
    for (int i = 0; i < n; ++i) {
        double Jc[3 * N], Jr[3 * N], IJ[3 * N];
        point_jacobian(n, R, p, i, &c[i * 3], Jc, Jr);
        /* IJ = Ibar_i J_r,i */
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < n; ++j) {
                double s = 0;
                for (int b = 0; b < 3; ++b) s += Iw[i * 9 + a * 3 + b] * Jr[b * n + j];
                IJ[a * n + j] = s;
            }
        for (int r = 0; r < n; ++r)
            for (int s = 0; s < n; ++s) {
                double acc = 0;
                for (int a = 0; a < 3; ++a)
                    acc += Jr[a * n + r] * IJ[a * n + s] +
                           rb->link[i].mass * Jc[a * n + r] * Jc[a * n + s];
                M[r * n + s] += acc;
            }
    }
    for (int j = 0; j < n; ++j) M[j * n + j] += rb->link[j].armature;
}

/* ------------------------------------------------------------------ */
/* h(q, qd) with the same accumulation as Eq. (8), from the link      */
/* Jacobians and their time derivatives (Sec. III-A):                 */
/*   h = sum_i m_i J_c,i^T (Jdot_c,i qd - g)                          */
/*         + J_r,i^T (Ibar_i Jdot_r,i qd + w_i x Ibar_i w_i)          */
/* Jdot columns: d/dt z_j = w_{j} x z_j,                              */
/*   d/dt [z_j x (c_i - p_j)] = zdot_j x (c_i - p_j)                  */
/*                              + z_j x (cdot_i - pdot_j).            */
/* ------------------------------------------------------------------ */
void ora_bias_jacobian(const ora_robot* rb, const double* q, const double* qd,
                       double* h)
{
    int n = rb->n;
    double R[N * 9], p[N * 3], c[N * 3], Iw[N * 9];
    double z[N * 3], w[N * 3], zdot[N * 3], pdot[N * 3];
    ora_fk(rb, q, R, p, NULL, NULL);
    link_world_inertial(rb, R, p, c, Iw);
    for (int j = 0; j < n; ++j) axis_of(R, j, &z[j * 3]);
    /* angular velocity of each link frame */
    for (int j = 0; j < n; ++j)
        for (int a = 0; a < 3; ++a)
            w[j * 3 + a] = (j ? w[(j - 1) * 3 + a] : 0.0) + z[j * 3 + a] * qd[j];
    for (int j = 0; j < n; ++j) v3_cross(&w[j * 3], &z[j * 3], &zdot[j * 3]);
    /* velocity of each joint origin (moves with the parent link) */
    for (int j = 0; j < n; ++j) {
        double acc[3] = {0, 0, 0};
        for (int k = 0; k < j; ++k) {
            double d[3], cr[3];
            for (int a = 0; a < 3; ++a) d[a] = p[j * 3 + a] - p[k * 3 + a];
            v3_cross(&z[k * 3], d, cr);
            for (int a = 0; a < 3; ++a) acc[a] += cr[a] * qd[k];
        }
        memcpy(&pdot[j * 3], acc, sizeof acc);
    }
    for (int r = 0; r < n; ++r) h[r] = 0;
    for (int i = 0; i < n; ++i) {
        const ora_link* L = &rb->link[i];
        double cdot[3] = {0, 0, 0};
        for (int k = 0; k <= i; ++k) {
            double d[3], cr[3];
            for (int a = 0; a < 3; ++a) d[a] = c[i * 3 + a] - p[k * 3 + a];
            v3_cross(&z[k * 3], d, cr);
            for (int a = 0; a < 3; ++a) cdot[a] += cr[a] * qd[k];
        }
        /* Jdot_c,i qd and Jdot_r,i qd */
        double jcq[3] = {0, 0, 0}, jrq[3] = {0, 0, 0};
        for (int j = 0; j <= i; ++j) {
            double d[3], t1[3], t2[3], dv[3];
            for (int a = 0; a < 3; ++a) {
                d[a] = c[i * 3 + a] - p[j * 3 + a];
                dv[a] = cdot[a] - pdot[j * 3 + a];
            }
            v3_cross(&zdot[j * 3], d, t1);
            v3_cross(&z[j * 3], dv, t2);
            for (int a = 0; a < 3; ++a) {
                jcq[a] += (t1[a] + t2[a]) * qd[j];
                jrq[a] += zdot[j * 3 + a] * qd[j];
            }
        }
        double lin[3], Iw_w[3], gyro[3], Ijr[3], ang[3];
        for (int a = 0; a < 3; ++a) lin[a] = L->mass * (jcq[a] - rb->gravity[a]);
        m3_vec(&Iw[i * 9], &w[i * 3], Iw_w);
        v3_cross(&w[i * 3], Iw_w, gyro);
        m3_vec(&Iw[i * 9], jrq, Ijr);
        for (int a = 0; a < 3; ++a) ang[a] = Ijr[a] + gyro[a];
        /* project: J_c,i^T lin + J_r,i^T ang */
        for (int j = 0; j <= i; ++j) {
            double d[3], cr[3];
            for (int a = 0; a < 3; ++a) d[a] = c[i * 3 + a] - p[j * 3 + a];
            v3_cross(&z[j * 3], d, cr);
            h[j] += v3_dot(cr, lin) + v3_dot(&z[j * 3], ang);
        }
    }
}

/* ------------------------------------------------------------------ */
/* spatial algebra (Featherstone, [angular; linear], link coordinates) */
/* used only by the CRBA / RNEA / ABA pins                             */
/* ------------------------------------------------------------------ */
/* motion transform from frame i-1 to frame i */
static void xup_of(const ora_link* L, double q, double* X)
{
    double Rz[9], Q[9], E[9], rx[9], Erx[9];
    rotz(q, Rz);
    m3_mul(L->R_parent, Rz, Q);
    m3_transpose(Q, E);
    skew(L->r_parent, rx);
    m3_mul(E, rx, Erx);
    m6_zero(X);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            X[a * 6 + b] = E[a * 3 + b];
            X[(3 + a) * 6 + 3 + b] = E[a * 3 + b];
            X[(3 + a) * 6 + b] = -Erx[a * 3 + b];
        }
}
/* spatial inertia about the link-frame origin */
static void spatial_inertia(const ora_link* L, double* I6)
{
    double Ic[9], cx[9], cxcxT[9];
    sym3(L->inertia, Ic);
    skew(L->com, cx);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += cx[a * 3 + k] * cx[b * 3 + k];
            cxcxT[a * 3 + b] = s;
        }
    m6_zero(I6);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            I6[a * 6 + b] = Ic[a * 3 + b] + L->mass * cxcxT[a * 3 + b];
            I6[a * 6 + 3 + b] = L->mass * cx[a * 3 + b];
            I6[(3 + a) * 6 + b] = L->mass * cx[b * 3 + a];
            I6[(3 + a) * 6 + 3 + b] = (a == b) ? L->mass : 0.0;
        }
}
static void crm(const double* v, double* X)
{
    double wx[9], vx[9];
    skew(v, wx);
    skew(v + 3, vx);
    m6_zero(X);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            X[a * 6 + b] = wx[a * 3 + b];
            X[(3 + a) * 6 + 3 + b] = wx[a * 3 + b];
            X[(3 + a) * 6 + b] = vx[a * 3 + b];
        }
}
static void crf(const double* v, double* X)
{
    double C[36];
    crm(v, C);
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) X[a * 6 + b] = -C[b * 6 + a];
}
/* world EE wrench [F; N] at p_ee -> spatial force on the last link */
static void ee_wrench_local(const ora_robot* rb, const double* q,
                            const double* f_ee, double* f6)
{
    double R[N * 9], p[N * 3];
    double Fl[3], Nl[3], m[3];
    ora_fk(rb, q, R, p, NULL, NULL);
    const double* Rn = &R[(rb->n - 1) * 9];
    m3_tvec(Rn, f_ee, Fl);
    m3_tvec(Rn, f_ee + 3, Nl);
    v3_cross(rb->r_ee, Fl, m);
    for (int a = 0; a < 3; ++a) { f6[a] = Nl[a] + m[a]; f6[3 + a] = Fl[a]; }
}

void ora_rnea(const ora_robot* rb, const double* q, const double* qd,
              const double* qdd, const double* f_ee, double* tau)
{
    int n = rb->n;
    double X[N][36], v[N][6], a[N][6], f[N][6];
    double fext[6] = {0, 0, 0, 0, 0, 0};
    if (f_ee) ee_wrench_local(rb, q, f_ee, fext);
    for (int i = 0; i < n; ++i) {
        double I6[36], Iv[6], Ia[6], cv[36], t[6];
        double vp[6] = {0, 0, 0, 0, 0, 0};
        double ap[6] = {0, 0, 0, -rb->gravity[0], -rb->gravity[1], -rb->gravity[2]};
        if (i) { memcpy(vp, v[i - 1], sizeof vp); memcpy(ap, a[i - 1], sizeof ap); }
        xup_of(&rb->link[i], q[i], X[i]);
        m6_vec(X[i], vp, v[i]);
        v[i][2] += qd[i];
        m6_vec(X[i], ap, a[i]);
        a[i][2] += qdd[i];
        {   /* + v_i x S qd_i */
            double s[6] = {0, 0, qd[i], 0, 0, 0};
            crm(v[i], cv);
            m6_vec(cv, s, t);
            for (int k = 0; k < 6; ++k) a[i][k] += t[k];
        }
        spatial_inertia(&rb->link[i], I6);
        m6_vec(I6, v[i], Iv);
        m6_vec(I6, a[i], Ia);
        crf(v[i], cv);
        m6_vec(cv, Iv, t);
        for (int k = 0; k < 6; ++k) f[i][k] = Ia[k] + t[k];
        if (i == n - 1)
            for (int k = 0; k < 6; ++k) f[i][k] -= fext[k];
    }
    for (int i = n - 1; i >= 0; --i) {
        tau[i] = f[i][2] + rb->link[i].armature * qdd[i];
        if (i) {
            double t[6];
            m6_tvec(X[i], f[i], t);
            for (int k = 0; k < 6; ++k) f[i - 1][k] += t[k];
        }
    }
}

void ora_crba(const ora_robot* rb, const double* q, double* M)
{
    int n = rb->n;
    double X[N][36], IC[N][36];
    for (int i = 0; i < n; ++i) {
        xup_of(&rb->link[i], q[i], X[i]);
        spatial_inertia(&rb->link[i], IC[i]);
    }
    for (int i = n - 1; i > 0; --i) {
        double T[36], U[36];
        m6_mul(IC[i], X[i], T);
        m6_tmul(X[i], T, U);
        for (int k = 0; k < 36; ++k) IC[i - 1][k] += U[k];
    }
    for (int i = 0; i < n; ++i) {
        double F[6];
        for (int k = 0; k < 6; ++k) F[k] = IC[i][k * 6 + 2];
        M[i * n + i] = F[2] + rb->link[i].armature;
        for (int j = i; j > 0; --j) {
            double t[6];
            m6_tvec(X[j], F, t);
            memcpy(F, t, sizeof t);
            M[i * n + (j - 1)] = M[(j - 1) * n + i] = F[2];
        }
    }
}

void ora_aba(const ora_robot* rb, const double* q, const double* qd,
             const double* tau, const double* f_ee, double* qdd)
{
    int n = rb->n;
    double X[N][36], v[N][6], c[N][6], IA[N][36], pA[N][6];
    double U[N][6], D[N], u[N];
    double fext[6] = {0, 0, 0, 0, 0, 0};
    if (f_ee) ee_wrench_local(rb, q, f_ee, fext);
    for (int i = 0; i < n; ++i) {
        double vp[6] = {0, 0, 0, 0, 0, 0}, cv[36], Iv[6], t[6];
        double s[6] = {0, 0, qd[i], 0, 0, 0};
        if (i) memcpy(vp, v[i - 1], sizeof vp);
        xup_of(&rb->link[i], q[i], X[i]);
        m6_vec(X[i], vp, v[i]);
        v[i][2] += qd[i];
        crm(v[i], cv);
        m6_vec(cv, s, c[i]);
        spatial_inertia(&rb->link[i], IA[i]);
        m6_vec(IA[i], v[i], Iv);
        crf(v[i], cv);
        m6_vec(cv, Iv, t);
        for (int k = 0; k < 6; ++k) pA[i][k] = t[k];
        if (i == n - 1)
            for (int k = 0; k < 6; ++k) pA[i][k] -= fext[k];
    }
    for (int i = n - 1; i >= 0; --i) {
        for (int k = 0; k < 6; ++k) U[i][k] = IA[i][k * 6 + 2];
        D[i] = U[i][2] + rb->link[i].armature;
        u[i] = tau[i] - pA[i][2];
        if (i) {
            double Ia[36], pa[6], Iac[6], T[36], W[36], t[6];
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b)
                    Ia[a * 6 + b] = IA[i][a * 6 + b] - U[i][a] * U[i][b] / D[i];
            m6_vec(Ia, c[i], Iac);
            for (int k = 0; k < 6; ++k) pa[k] = pA[i][k] + Iac[k] + U[i][k] * u[i] / D[i];
            m6_mul(Ia, X[i], T);
            m6_tmul(X[i], T, W);
            for (int k = 0; k < 36; ++k) IA[i - 1][k] += W[k];
            m6_tvec(X[i], pa, t);
            for (int k = 0; k < 6; ++k) pA[i - 1][k] += t[k];
        }
    }
    double a[N][6];
    for (int i = 0; i < n; ++i) {
        double ap[6] = {0, 0, 0, -rb->gravity[0], -rb->gravity[1], -rb->gravity[2]};
        double ai[6];
        if (i) memcpy(ap, a[i - 1], sizeof ap);
        m6_vec(X[i], ap, ai);
        for (int k = 0; k < 6; ++k) ai[k] += c[i][k];
        double Ua = 0;
        for (int k = 0; k < 6; ++k) Ua += U[i][k] * ai[k];
        qdd[i] = (u[i] - Ua) / D[i];
        ai[2] += qdd[i];
        memcpy(a[i], ai, sizeof ai);
    }
}

int ora_cholesky_solve(int n, const double* A, double* b)
{
    double L[N * N > 36 ? N * N : 36];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            if (i == j) {
                if (!(s > 0)) return ORA_ESINGULAR;
                L[i * n + i] = sqrt(s);
            } else {
                L[i * n + j] = s / L[j * n + j];
            }
        }
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
        b[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
        b[i] = s / L[i * n + i];
    }
    return ORA_OK;
}

/* Eq. (6): qdd = M^-1 (tau + tau_ext - h), with tau_ext = J^T F_ext
   (Sec. III-A) for the given EE wrench. */
int ora_forward_dynamics(const ora_robot* rb, const double* q,
                         const double* qd, const double* tau,
                         const double* f_ee, double* qdd)
{
    int n = rb->n;
    double M[N * N], h[N];
    ora_mass_jacobian_sum(rb, q, M);
    ora_bias_jacobian(rb, q, qd, h);
    for (int j = 0; j < n; ++j) qdd[j] = tau[j] - h[j];
    if (f_ee) {
        double J[6 * N];
        ora_ee_jacobian(rb, q, J);
        for (int j = 0; j < n; ++j)
            for (int r = 0; r < 6; ++r) qdd[j] += J[r * n + j] * f_ee[r];
    }
    return ora_cholesky_solve(n, M, qdd);
}

double ora_energy(const ora_robot* rb, const double* q, const double* qd)
{
    int n = rb->n;
    double M[N * N], R[N * 9], p[N * 3], c[N * 3], Iw[N * 9];
    ora_mass_jacobian_sum(rb, q, M);
    double T = 0;
    for (int r = 0; r < n; ++r)
        for (int s = 0; s < n; ++s) T += 0.5 * qd[r] * M[r * n + s] * qd[s];
    ora_fk(rb, q, R, p, NULL, NULL);
    link_world_inertial(rb, R, p, c, Iw);
    double V = 0;
    for (int i = 0; i < n; ++i) V -= rb->link[i].mass * v3_dot(rb->gravity, &c[i * 3]);
    return T + V;
}

/* ------------------------------------------------------------------ */
/* task space                                                          */
/* ------------------------------------------------------------------ */
void ora_quat_to_R(const double* quat, double* R)
{
    double w = quat[0], x = quat[1], y = quat[2], z = quat[3];
    double nrm = sqrt(w * w + x * x + y * y + z * z);
    w /= nrm; x /= nrm; y /= nrm; z /= nrm;
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* Rotation vector rho with |rho| = theta in [0, pi] (Eq. 11's log map).
   theta = atan2(|vee(R - R^T)|/2, (tr R - 1)/2).  Near pi the axis comes
   from the symmetric part; the sign there is immaterial to the quadratic
   cost. */
void ora_so3_log(const double* R, double* rho)
{
    double vee[3] = {R[7] - R[5], R[2] - R[6], R[3] - R[1]};
    double s = 0.5 * sqrt(v3_dot(vee, vee));
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    double th = atan2(s, c);
    if (s < 1e-7 && c < 0) {
        double B[9];
        for (int a = 0; a < 9; ++a) B[a] = 0.5 * (R[a] + R[(a % 3) * 3 + a / 3]);
        for (int a = 0; a < 3; ++a) B[a * 4] -= c;
        int m = 0;
        for (int a = 1; a < 3; ++a) if (B[a * 4] > B[m * 4]) m = a;
        double den = sqrt(B[m * 4] * (1.0 - c));
        double ax[3] = {B[m] / den, B[3 + m] / den, B[6 + m] / den};
        if (v3_dot(ax, vee) < 0) for (int a = 0; a < 3; ++a) ax[a] = -ax[a];
        for (int a = 0; a < 3; ++a) rho[a] = th * ax[a];
        return;
    }
    double f = (s > 1e-12) ? th / s : 1.0; /* theta / sin(theta) */
    for (int a = 0; a < 3; ++a) rho[a] = 0.5 * f * vee[a];
}

/* Eq. (13): F_ee = Jbar^T tau_F with Jbar = M^-1 J^T (J M^-1 J^T)^-1,
   i.e. F_ee = Lambda J M^-1 tau_F, Lambda = (J M^-1 J^T)^-1. */
int ora_force_estimate(const ora_robot* rb, const double* q,
                       const double* tau_F, double* F_ee)
{
    int n = rb->n;
    double M[N * N], J[6 * N], Y[N * 6], A[36], b[6], x[N];
    ora_mass_jacobian_sum(rb, q, M);
    ora_ee_jacobian(rb, q, J);
    for (int r = 0; r < 6; ++r) {       /* column r of Y = M^-1 J^T */
        double col[N];
        for (int j = 0; j < n; ++j) col[j] = J[r * n + j];
        if (ora_cholesky_solve(n, M, col)) return ORA_ESINGULAR;
        for (int j = 0; j < n; ++j) Y[j * 6 + r] = col[j];
    }
    for (int r = 0; r < 6; ++r)
        for (int s = 0; s < 6; ++s) {
            double acc = 0;
            for (int j = 0; j < n; ++j) acc += J[r * n + j] * Y[j * 6 + s];
            A[r * 6 + s] = acc;
        }
    for (int j = 0; j < n; ++j) x[j] = tau_F[j];
    if (ora_cholesky_solve(n, M, x)) return ORA_ESINGULAR;
    for (int r = 0; r < 6; ++r) {
        double acc = 0;
        for (int j = 0; j < n; ++j) acc += J[r * n + j] * x[j];
        b[r] = acc;
    }
    if (ora_cholesky_solve(6, A, b)) return ORA_ESINGULAR;
    memcpy(F_ee, b, sizeof b);
    return ORA_OK;
}

/* Wall model (planar, unilateral spring-damper at the EE point, force along
   the normal, never pulling): delta = d0 - n.p, F = n max(0, k delta +
   c d(delta)/dt).  A workload convention: the paper gives no contact
   model. */
void ora_wall_force(const ora_cost* cp, const double* p_ee,
                    const double* v_ee, double* F)
{
    double delta = cp->wall_d0 - v3_dot(cp->wall_n, p_ee);
    double ddelta = -v3_dot(cp->wall_n, v_ee);
    double mag = cp->wall_k * delta + cp->wall_c * ddelta;
    if (mag < 0) mag = 0;
    for (int a = 0; a < 3; ++a) F[a] = cp->wall_n[a] * mag;
}

/* EE wrench acting on the robot from the environment at state (q, qd). */
static void ext_wrench(const ora_robot* rb, const ora_cost* cp, const double* q,
                       const double* qd, double* f)
{
    int n = rb->n;
    for (int a = 0; a < 6; ++a) f[a] = 0;
    if (cp->ext_mode == ORA_EXT_CONST) {
        for (int a = 0; a < 6; ++a) f[a] = cp->F_ext[a];
    } else if (cp->ext_mode == ORA_EXT_WALL) {
        double J[6 * N], pe[3], R[N * 9], p[N * 3], ve[3] = {0, 0, 0};
        ora_fk(rb, q, R, p, pe, NULL);
        ora_ee_jacobian(rb, q, J);
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < n; ++j) ve[a] += J[a * n + j] * qd[j];
        ora_wall_force(cp, pe, ve, f);
    }
}

/* ------------------------------------------------------------------ */
/* noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the   */
/* Box-Muller transform (1958); counter (c, t, k, tick), key = seed.  */
/* Eq. (2): delta u ~ N(0, Sigma_u), Sigma_u = diag(sigma^2).         */
/* ------------------------------------------------------------------ */
void ora_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                       uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void ora_normals(uint64_t seed, uint64_t tick, uint32_t k, uint32_t t,
                 double z[8])
{
    const double two32 = 4294967296.0;
    const double pi = 3.14159265358979323846;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint32_t call = 0; call < 2; ++call) {
        uint32_t ctr[4] = {call, t, k, (uint32_t)tick}, x[4];
        ora_philox4x32_10(ctr, key, x);
        for (int pr = 0; pr < 2; ++pr) {
            double ua = ((double)x[2 * pr] + 1.0) / two32; /* (0, 1] */
            double ub = (double)x[2 * pr + 1] / two32;     /* [0, 1) */
            double r = sqrt(-2.0 * log(ua));
            z[call * 4 + pr * 2 + 0] = r * cos(2.0 * pi * ub);
            z[call * 4 + pr * 2 + 1] = r * sin(2.0 * pi * ub);
        }
    }
}

/* ------------------------------------------------------------------ */
/* costs (Eqs. 9-14)                                                   */
/* ------------------------------------------------------------------ */
static double hinge_sq(double x) { return x > 0 ? x * x : 0.0; }

static int any_nonzero(const double* w, int m)
{
    for (int i = 0; i < m; ++i) if (w[i] != 0.0) return 1;
    return 0;
}

/* C_motion, Eq. (11): e_p^T W_pos e_p + rho^T W_ori rho,
   rho = log(R_des^T R_ee); W diagonal (axis selection). */
static void motion_cost(const ora_robot* rb, const ora_cost* cp,
                        const ora_target* tg, const double* q,
                        double* cpos, double* cori)
{
    double R[N * 9], p[N * 3], pe[3], Re[9], Rd[9], Rdt[9], Rerr[9], rho[3];
    ora_fk(rb, q, R, p, pe, Re);
    *cpos = 0;
    for (int a = 0; a < 3; ++a) {
        double e = tg->p_des[a] - pe[a];
        *cpos += cp->W_pos[a] * e * e;
    }
    *cori = 0;
    if (any_nonzero(cp->W_ori, 3)) {
        ora_quat_to_R(tg->quat_des, Rd);
        m3_transpose(Rd, Rdt);
        m3_mul(Rdt, Re, Rerr);
        ora_so3_log(Rerr, rho);
        for (int a = 0; a < 3; ++a) *cori += cp->W_ori[a] * rho[a] * rho[a];
    }
}

/* C_joint (Eq. 14 first term; its exact form is deferred by the paper to
   another work): squared hinge on position and speed limits plus a posture
   term w_post |q - q_rest|^2. */
static double joint_cost(const ora_robot* rb, const ora_cost* cp,
                         const double* q, const double* qd)
{
    double s = 0;
    for (int j = 0; j < rb->n; ++j) {
        const ora_link* L = &rb->link[j];
        double d = q[j] - cp->q_rest[j];
        s += cp->w_q * (hinge_sq(q[j] - L->q_max) + hinge_sq(L->q_min - q[j]));
        s += cp->w_qd * hinge_sq(fabs(qd[j]) - L->qd_max);
        s += cp->w_post * d * d;
    }
    return s;
}

double ora_running_cost(const ora_robot* rb, const ora_cost* cp,
                        const ora_target* tg, const double* q,
                        const double* qd, const double* v, double* parts)
{
    int n = rb->n;
    double cpos, cori, cforce = 0, cjoint, ctau = 0;
    motion_cost(rb, cp, tg, q, &cpos, &cori);
    if (any_nonzero(cp->W_force, 6) || any_nonzero(cp->W_reg, 6)) {
        /* Eq. (12) with F_ee from Eq. (13) */
        double tauF[N], F[6];
        for (int j = 0; j < n; ++j) tauF[j] = v[j];
        if (cp->force_mode == 0) {
            double g[N], zero[N] = {0};
            ora_bias_jacobian(rb, q, zero, g); /* h(q, 0) = g(q) */
            for (int j = 0; j < n; ++j) tauF[j] -= g[j];
        }
        if (ora_force_estimate(rb, q, tauF, F)) {
            cforce = NAN;
        } else {
            for (int a = 0; a < 6; ++a) {
                double e = tg->F_des[a] - F[a];
                cforce += cp->W_force[a] * e * e + cp->W_reg[a] * F[a] * F[a];
            }
        }
    }
    cjoint = joint_cost(rb, cp, q, qd);
    for (int j = 0; j < n; ++j)
        ctau += cp->w_tau * hinge_sq(fabs(v[j]) - rb->link[j].tau_max);
    /* Eq. (14): C_constraint = C_joint + C_collision */
    double ccoll = ora_collision_cost(rb, cp, q, NULL);
    double total = cpos + cori + cforce + cjoint + ctau + ccoll;
    if (parts) {
        parts[0] = cpos; parts[1] = cori; parts[2] = cforce;
        parts[3] = cjoint; parts[4] = ctau; parts[5] = ccoll; parts[6] = total;
    }
    return total;
}

/* Minimum distance between two segments (the quantity Eq. (15) thresholds;
   the paper computes it with Lumelsky's method).  Here straight from the
   definition: |a0 + s da - b0 - t db|^2 is a convex quadratic in (s, t), so
   its minimum over the unit square is the interior stationary point when
   that lies in the square, else the minimum over the four edges, each a
   one-variable quadratic minimised by clamping its stationary point. */
static double seg_d2(const double* a0, const double* da, const double* b0, const double* db, double s, double t)
{
    double d2 = 0;
    for (int c = 0; c < 3; ++c) {
        double e = a0[c] + s * da[c] - b0[c] - t * db[c];
        d2 += e * e;
    }
    return d2;
}

static double clamp01(double x) { return x < 0 ? 0 : (x > 1 ? 1 : x); }

double ora_segment_distance(const double* a0, const double* a1, const double* b0, const double* b1)
{
    double da[3], db[3], r[3];
    for (int c = 0; c < 3; ++c) { da[c] = a1[c] - a0[c]; db[c] = b1[c] - b0[c]; r[c] = a0[c] - b0[c]; }
    /* f(s,t) = |r + s da - t db|^2 = A s^2 - 2 B s t + E t^2 + 2 C s - 2 F t + |r|^2 */
    double A = 0, B = 0, E = 0, Cc = 0, F = 0;
    for (int c = 0; c < 3; ++c) {
        A += da[c] * da[c]; B += da[c] * db[c]; E += db[c] * db[c];
        Cc += da[c] * r[c]; F += db[c] * r[c];
    }
    double best = INFINITY;
    double det = A * E - B * B;
    if (det > 1e-12 * (A * E + 1e-300)) {
        /* grad = 0:  A s - B t = -C,  -B s + E t = F */
        double s = (-Cc * E + B * F) / det, t = (A * F - B * Cc) / det;
        if (s >= 0 && s <= 1 && t >= 0 && t <= 1) best = seg_d2(a0, da, b0, db, s, t);
    }
    /* edges s = 0, 1: minimise over t; edges t = 0, 1: minimise over s */
    for (int e = 0; e < 2; ++e) {
        double s = e, t = E > 0 ? clamp01((F + B * s) / E) : 0;
        double d2 = seg_d2(a0, da, b0, db, s, t);
        if (d2 < best) best = d2;
        t = e;
        s = A > 0 ? clamp01((B * t - Cc) / A) : 0;
        d2 = seg_d2(a0, da, b0, db, s, t);
        if (d2 < best) best = d2;
    }
    return sqrt(best);
}

void ora_link_segments(const ora_robot* rb, const double* q, double* seg)
{
    int n = rb->n;
    double R[9 * N], p[3 * N], pe[3], Re[9];
    ora_fk(rb, q, R, p, pe, Re);
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            seg[i * 6 + c] = p[i * 3 + c];
            seg[i * 6 + 3 + c] = i + 1 < n ? p[(i + 1) * 3 + c] : pe[c];
        }
}

double ora_collision_cost(const ora_robot* rb, const ora_cost* cp, const double* q, double* margin)
{
    double m = INFINITY, cost = 0;
    if (cp->n_pairs > 0) {
        int n = rb->n;
        double seg[6 * (N + ORA_MAXOBS)];
        ora_link_segments(rb, q, seg);
        for (int o = 0; o < cp->n_obstacles; ++o)
            for (int c = 0; c < 6; ++c) seg[(n + o) * 6 + c] = cp->obstacles[o][c];
        for (int i = 0; i < cp->n_pairs; ++i) {
            const double* a = seg + 6 * cp->pairs[i][0];
            const double* b = seg + 6 * cp->pairs[i][1];
            double d = ora_segment_distance(a, a + 3, b, b + 3);
            if (d < cp->d_th[i]) cost += cp->w_collision;   /* the indicator of Eq. (15) */
            if (fabs(d - cp->d_th[i]) < m) m = fabs(d - cp->d_th[i]);
        }
    }
    if (margin) *margin = m;
    return cost;
}

/* phi(x_T): the paper leaves it unspecified; here w_T times the motion and
   joint terms at the final state. */
double ora_terminal_cost(const ora_robot* rb, const ora_cost* cp,
                         const ora_target* tg, const double* q,
                         const double* qd)
{
    double cpos, cori;
    motion_cost(rb, cp, tg, q, &cpos, &cori);
    return cp->w_terminal * (cpos + cori + joint_cost(rb, cp, q, qd));
}

/* ------------------------------------------------------------------ */
/* MPPI (Sec. II and Sec. III)                                        */
/* ------------------------------------------------------------------ */
/* One rollout: v_t = u_t + delta u_t (Eq. 2), qdd by Eq. (6) with the
   per-step M and h (Sec. III-A), semi-implicit Euler as written in
   Eq. (7), S = phi(x_T) + sum_t l(x_t, v_t) (Eq. 3). */
double ora_rollout(const ora_robot* rb, const ora_cost* cp,
                   const ora_target* tg, const double* q0, const double* qd0,
                   const double* U_nom, uint64_t seed, uint64_t tick,
                   uint32_t k, double* noise)
{
    return ora_rollout_margin(rb, cp, tg, q0, qd0, U_nom, seed, tick, k, noise, NULL);
}

double ora_rollout_margin(const ora_robot* rb, const ora_cost* cp,
                          const ora_target* tg, const double* q0, const double* qd0,
                          const double* U_nom, uint64_t seed, uint64_t tick,
                          uint32_t k, double* noise, double* margin)
{
    int n = rb->n;
    if (margin) *margin = INFINITY;
    double q[N], qd[N], S = 0.0;
    double tau_ext_const[N] = {0};
    memcpy(q, q0, sizeof(double) * n);
    memcpy(qd, qd0, sizeof(double) * n);
    if (cp->ext_mode == ORA_EXT_CONST) {
        /* tau_ext = J^T(q_0) F_ext, held for the whole horizon */
        double J[6 * N];
        ora_ee_jacobian(rb, q0, J);
        for (int j = 0; j < n; ++j)
            for (int r = 0; r < 6; ++r) tau_ext_const[j] += J[r * n + j] * cp->F_ext[r];
    }
    double du_prev[N] = {0};
    const double rho = cp->noise_rho, rho_c = sqrt(1.0 - cp->noise_rho * cp->noise_rho);
    for (int t = 0; t < cp->T; ++t) {
        double z[8], v[N], rhs[N], qdd[N];
        ora_normals(seed, tick, k, (uint32_t)t, z);
        for (int j = 0; j < n; ++j) {
            /* Eq. 2's perturbation; correlated in time when rho > 0 */
            double du = t == 0 ? cp->sigma[j] * z[j] : rho * du_prev[j] + rho_c * cp->sigma[j] * z[j];
            du_prev[j] = du;
            if (noise) noise[t * n + j] = du;
            v[j] = U_nom[t * n + j] + du;
        }
        S += ora_running_cost(rb, cp, tg, q, qd, v, NULL);
        if (margin && cp->n_pairs > 0) {
            double m;
            ora_collision_cost(rb, cp, q, &m);
            if (m < *margin) *margin = m;
        }
        for (int j = 0; j < n; ++j) rhs[j] = v[j] + tau_ext_const[j];
        if (cp->ext_mode == ORA_EXT_WALL) {
            double f[6];
            ext_wrench(rb, cp, q, qd, f);
            if (ora_forward_dynamics(rb, q, qd, rhs, f, qdd)) return INFINITY;
        } else {
            if (ora_forward_dynamics(rb, q, qd, rhs, NULL, qdd)) return INFINITY;
        }
        for (int j = 0; j < n; ++j) {
            qd[j] += qdd[j] * cp->dt;
            q[j] += qd[j] * cp->dt;
        }
    }
    S += ora_terminal_cost(rb, cp, tg, q, qd);
    return isfinite(S) ? S : INFINITY;
}

/* Eq. (4a)/(4b) with the minimum-cost shift: omega_k = exp(-(S_k - S_min)
   / lambda), u*_t <- u_t + sum_k omega_k du_k,t / sum_k omega_k.  A
   non-finite S_k gets omega_k = 0; if no S_k is finite U_new = U_nom. */
int ora_weights_update(int K, int T, int n, double lambda, const double* S,
                       const double* noise, const double* U_nom,
                       double* U_new, double* weights)
{
    double Smin = INFINITY;
    for (int k = 0; k < K; ++k)
        if (isfinite(S[k]) && S[k] < Smin) Smin = S[k];
    if (!isfinite(Smin)) {
        for (int i = 0; i < T * n; ++i) U_new[i] = U_nom[i];
        if (weights) for (int k = 0; k < K; ++k) weights[k] = 0;
        return ORA_ENONFINITE;
    }
    double* w = (double*)malloc(sizeof(double) * K);
    if (!w) return ORA_EINVAL;
    double eta = 0;
    for (int k = 0; k < K; ++k) {
        w[k] = isfinite(S[k]) ? exp(-(S[k] - Smin) / lambda) : 0.0;
        if (weights) weights[k] = w[k];
        eta += w[k];
    }
    for (int i = 0; i < T * n; ++i) {
        double acc = 0;
        for (int k = 0; k < K; ++k) acc += w[k] * noise[(size_t)k * T * n + i];
        U_new[i] = U_nom[i] + acc / eta;
    }
    free(w);
    return ORA_OK;
}

int ora_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int ora_update(const ora_robot* rb, const ora_cost* cp, const ora_target* tg,
               const double* q0, const double* qd0, const double* U_nom,
               uint64_t seed, uint64_t tick, double* U_new, double* costs,
               double* noise, int nthreads)
{
    if (!rb || !cp || !tg || !q0 || !qd0 || !U_nom || !U_new) return ORA_EINVAL;
    if (rb->n < 1 || rb->n > ORA_MAXJ || cp->K < 1 || cp->T < 1 ||
        !(cp->dt > 0) || !(cp->lambda > 0))
        return ORA_EINVAL;
    int K = cp->K, T = cp->T, n = rb->n;
    size_t per = (size_t)T * n;
    double* S = costs;
    double* E = noise;
    int ownS = 0, ownE = 0;
    if (!S) { S = (double*)malloc(sizeof(double) * K); ownS = 1; }
    if (!E) { E = (double*)malloc(sizeof(double) * per * K); ownE = 1; }
    if (!S || !E) {
        if (ownS) free(S);
        if (ownE) free(E);
        return ORA_EINVAL;
    }
    int iters = cp->iterations > 1 ? cp->iterations : 1;
    double* Ucur = (double*)malloc(sizeof(double) * per);
    if (!Ucur) {
        if (ownS) free(S);
        if (ownE) free(E);
        return ORA_EINVAL;
    }
    memcpy(Ucur, U_nom, sizeof(double) * per);
    int st = ORA_OK;
    for (int it = 0; it < iters; ++it) {
        uint64_t tk = tick * (uint64_t)iters + (uint64_t)it;
#ifdef _OPENMP
        int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nt)
#endif
        for (int k = 0; k < K; ++k)
            S[k] = ora_rollout(rb, cp, tg, q0, qd0, Ucur, seed, tk,
                               (uint32_t)k, E + per * (size_t)k);
        st = ora_weights_update(K, T, n, cp->lambda, S, E, Ucur, U_new, NULL);
        memcpy(Ucur, U_new, sizeof(double) * per);
    }
    (void)nthreads;
    free(Ucur);
    if (ownS) free(S);
    if (ownE) free(E);
    return st;
}

/* Warm start after s horizon steps of elapsed time (the receding horizon
   at the end of Sec. II, for a solver period that differs from dt): the
   plan U is read as piecewise constant (row i held over [i, i + 1) in
   steps, the last row held past the horizon) and row t of out is its mean
   over [t + s, t + s + 1). */
void ora_warm_start(int T, int n, const double* U, double s, double* out)
{
    for (int t = 0; t < T; ++t) {
        const double a = t + s, b = a + 1.0;
        for (int j = 0; j < n; ++j) out[t * n + j] = 0.0;
        /* overlap of [a, b) with each held interval [i, i + 1) */
        const int i0 = (int)floor(a);
        for (int i = i0; i <= i0 + 1; ++i) {
            const double lo = a > i ? a : (double)i;
            const double hi = b < i + 1.0 ? b : i + 1.0;
            if (hi <= lo) continue;
            const int row = i < T ? i : T - 1;
            for (int j = 0; j < n; ++j) out[t * n + j] += (hi - lo) * U[row * n + j];
        }
    }
}

/* Plant for the closed loop: the command is held (zero-order hold) over
   one control period, split into semi-implicit Euler substeps, with the
   torque clamped to the joint limits. */
void ora_plant_step(const ora_robot* rb, const ora_cost* cp, double* q,
                    double* qd, const double* u, double dt, int substeps)
{
    int n = rb->n;
    double h = dt / substeps, tau[N];
    for (int j = 0; j < n; ++j) {
        double lim = rb->link[j].tau_max;
        tau[j] = u[j] > lim ? lim : (u[j] < -lim ? -lim : u[j]);
    }
    for (int s = 0; s < substeps; ++s) {
        double f[6], qdd[N];
        ext_wrench(rb, cp, q, qd, f);
        ora_forward_dynamics(rb, q, qd, tau, f, qdd);
        for (int j = 0; j < n; ++j) {
            qd[j] += qdd[j] * h;
            q[j] += qd[j] * h;
        }
    }
}
