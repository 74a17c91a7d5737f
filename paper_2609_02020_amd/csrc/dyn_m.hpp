// dyn_m.hpp -- the paper's own dynamics route for one rollout step, the
// alternative to the articulated-body step of dyn.hpp (Sec. III-A):
//   * M formed per step as the Jacobian sum of Eq. 8,
//       M = sum_i (m_i J_v,i^T J_v,i + J_w,i^T Ibar_i J_w,i) + diag(a),
//     with J_v,i, J_w,i the CoM Jacobians of link i (world axes) and
//     Ibar_i = R_i I_i R_i^T;
//   * h = sum_i (J_v,i^T m_i (Jdot_v,i qd - g) + J_w,i^T (Ibar_i Jdot_w,i qd
//     + w_i x Ibar_i w_i)), where Jdot_i qd is the CoM (angular)
//     acceleration at zero joint acceleration, propagated link by link, and
//     the J^T products are accumulated from the tip;
//   * qdd = M^-1 (tau + tau_ext - h) (Eq. 6) by a 7x7 Cholesky solve;
//   * when the force cost is on, F_ee = (J M^-1 J^T)^-1 J M^-1 tau_F
//     (Eq. 13) with J the EE Jacobian [J_v; J_w] at the EE point: with the
//     Cholesky factor M = L L^T, seven forward substitutions give
//     A^T = L^-1 J^T and y = L^-1 tau_F, and F_ee is the least-squares
//     solution of A^T x = y (lsq_wrench of dyn.hpp).
// Same inputs and outputs as dyn_step (StepOut: qdd, EE pose, F_ee).
#pragma once

#include "dyn.hpp"

namespace mppi {

// In-place lower Cholesky factor of the symmetric positive definite A (the
// lower triangle is read); idg receives the reciprocal diagonal.
template <int N, typename R> MPPI_HD void chol_lower(R (&A)[N][N], R (&idg)[N])
{
#pragma unroll
    for (int j = 0; j < N; ++j) {
        R d = A[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
        const R l = rsqrt_sqrt_(d);
        A[j][j] = l;
        idg[j] = rcp_(l);
#pragma unroll
        for (int i = j + 1; i < N; ++i) {
            R s = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= A[i][k] * A[j][k];
            A[i][j] = s * idg[j];
        }
    }
}

// x = (L L^T)^-1 b in place
template <int N, typename R> MPPI_HD void chol_solve(const R (&L)[N][N], const R (&idg)[N], R* b)
{
#pragma unroll
    for (int i = 0; i < N; ++i) {
        R s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * b[k];
        b[i] = s * idg[i];
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        R s = b[i];
#pragma unroll
        for (int k = i + 1; k < N; ++k) s -= L[k][i] * b[k];
        b[i] = s * idg[i];
    }
}

// Jacobian-transpose accumulation from the tip: out_j = z_j . (N_j - p_j x F_j)
// with F_j = sum_{i >= j} f_i and N_j = sum_{i >= j} (c_i x f_i + n_i),
// i.e. sum_i (J_v,i^T f_i + J_w,i^T n_i) for point forces f_i at c_i.
template <typename R>
MPPI_HD void jt_accumulate(const R (&z)[NJ][3], const R (&p)[NJ][3], const R (&cm)[NJ][3], const R (&f)[NJ][3],
                           const R (&n)[NJ][3], R* out)
{
    R Fs[3] = {R(0), R(0), R(0)}, Ns[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = NJ - 1; i >= 0; --i) {
        R cf[3], pF[3];
        cross3(cm[i], f[i], cf);
#pragma unroll
        for (int c = 0; c < 3; ++c) { Fs[c] += f[i][c]; Ns[c] += cf[c] + n[i][c]; }
        cross3(p[i], Fs, pF);
        out[i] = z[i][0] * (Ns[0] - pF[0]) + z[i][1] * (Ns[1] - pF[1]) + z[i][2] * (Ns[2] - pF[2]);
    }
}

template <typename R, bool FORCE>
MPPI_HD void dyn_step_m(const ModelM<R>& Mdl, const CostM<R>& Cst, int ext, const R* q, const R* qd,
                        const R* tau, const R* v, StepOut<R>& out)
{
    R z[NJ][3], p[NJ][3], cm[NJ][3], Ib[NJ][6];
    // ---- kinematics: joint axes, joint origins, CoMs, world inertias
    R Rw[9] = {R(1), R(0), R(0), R(0), R(1), R(0), R(0), R(0), R(1)};
    R pw[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const LinkM<R>& L = Mdl.L[i];
        R c, s, Q[9], d[3], cw[3];
        sincos_(q[i], &s, &c);
        joint_rot(L.Rp, c, s, Q);
        mv3(Rw, L.rp, d);
        pw[0] += d[0]; pw[1] += d[1]; pw[2] += d[2];
        mm3(Rw, Q, Rw);
        z[i][0] = Rw[2]; z[i][1] = Rw[5]; z[i][2] = Rw[8];
        p[i][0] = pw[0]; p[i][1] = pw[1]; p[i][2] = pw[2];
        mv3(Rw, L.com, cw);
        cm[i][0] = pw[0] + cw[0]; cm[i][1] = pw[1] + cw[1]; cm[i][2] = pw[2] + cw[2];
        congr_sym3<false>(Rw, L.Ic, Ib[i]);
    }
    R ree_w[3];
    mv3(Rw, Mdl.ree, ree_w);
    out.pee[0] = pw[0] + ree_w[0]; out.pee[1] = pw[1] + ree_w[1]; out.pee[2] = pw[2] + ree_w[2];
#pragma unroll
    for (int a = 0; a < 9; ++a) out.Rn[a] = Rw[a];

    // ---- velocities and zero-joint-acceleration terms (Jdot qd), link forces
    R f[NJ][3], nm[NJ][3];
    R w[3] = {R(0), R(0), R(0)}, al[3] = {R(0), R(0), R(0)};   // link i-1: omega, alpha (qdd = 0)
    R vp[3] = {R(0), R(0), R(0)}, ap[3] = {R(0), R(0), R(0)};  // origin of joint i-1: velocity, acceleration
    R pprev[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        // the origin of joint i moves with link i-1
        R r[3], t1[3], t2[3], t3[3];
        r[0] = p[i][0] - pprev[0]; r[1] = p[i][1] - pprev[1]; r[2] = p[i][2] - pprev[2];
        cross3(w, r, t1);
        cross3(al, r, t2);
        cross3(w, t1, t3);
#pragma unroll
        for (int c = 0; c < 3; ++c) { vp[c] += t1[c]; ap[c] += t2[c] + t3[c]; }
        // link i: omega_i = omega_{i-1} + z_i qd_i, alpha_i = alpha_{i-1} + omega_{i-1} x z_i qd_i
        const R wz[3] = {z[i][0] * qd[i], z[i][1] * qd[i], z[i][2] * qd[i]};
        R wxz[3];
        cross3(w, wz, wxz);
#pragma unroll
        for (int c = 0; c < 3; ++c) { al[c] += wxz[c]; w[c] += wz[c]; }
        // CoM acceleration at qdd = 0: a_p + alpha x d + omega x (omega x d)
        R dc[3] = {cm[i][0] - p[i][0], cm[i][1] - p[i][1], cm[i][2] - p[i][2]};
        R u1[3], u2[3], u3[3];
        cross3(al, dc, u1);
        cross3(w, dc, u2);
        cross3(w, u2, u3);
        const R m = Mdl.L[i].m;
#pragma unroll
        for (int c = 0; c < 3; ++c) f[i][c] = m * (ap[c] + u1[c] + u3[c] - Mdl.g[c]);
        // Ibar alpha + omega x (Ibar omega)
        const R* I = Ib[i];
        R Ia[3], Iw[3], wIw[3];
        Ia[0] = I[0] * al[0] + I[3] * al[1] + I[4] * al[2];
        Ia[1] = I[3] * al[0] + I[1] * al[1] + I[5] * al[2];
        Ia[2] = I[4] * al[0] + I[5] * al[1] + I[2] * al[2];
        Iw[0] = I[0] * w[0] + I[3] * w[1] + I[4] * w[2];
        Iw[1] = I[3] * w[0] + I[1] * w[1] + I[5] * w[2];
        Iw[2] = I[4] * w[0] + I[5] * w[1] + I[2] * w[2];
        cross3(w, Iw, wIw);
#pragma unroll
        for (int c = 0; c < 3; ++c) { nm[i][c] = Ia[c] + wIw[c]; pprev[c] = p[i][c]; }
    }
    R h[NJ];
    jt_accumulate(z, p, cm, f, nm, h);

    // ---- external torque at the EE point
    R tauext[NJ] = {R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
    if (ext == EXTW_WALL) {
        R rr[3] = {out.pee[0] - p[NJ - 1][0], out.pee[1] - p[NJ - 1][1], out.pee[2] - p[NJ - 1][2]};
        R wxr[3];
        // the EE point moves with the last link; vp is still joint n-1's origin velocity
        cross3(w, rr, wxr);
        const R vee[3] = {vp[0] + wxr[0], vp[1] + wxr[1], vp[2] + wxr[2]};
        const R delta = Cst.wall_d0 - dot3(Cst.wall_n, out.pee);
        const R ddelta = -dot3(Cst.wall_n, vee);
        const R mag = hinge(Cst.wall_k * delta + Cst.wall_c * ddelta);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            R rj[3] = {out.pee[0] - p[j][0], out.pee[1] - p[j][1], out.pee[2] - p[j][2]}, jv[3];
            cross3(z[j], rj, jv);
            tauext[j] = mag * dot3(jv, Cst.wall_n);
        }
    }

    // ---- M by Eq. 8 (lower triangle), then qdd
    R Mm[NJ][NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int k = 0; k < NJ; ++k) Mm[j][k] = (j == k) ? Mdl.L[j].arm : R(0);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const R m = Mdl.L[i].m;
        const R* I = Ib[i];
        R jv[NJ][3], Iz[NJ][3];
#pragma unroll
        for (int k = 0; k <= i; ++k) {
            R rk[3] = {cm[i][0] - p[k][0], cm[i][1] - p[k][1], cm[i][2] - p[k][2]};
            cross3(z[k], rk, jv[k]);
            Iz[k][0] = I[0] * z[k][0] + I[3] * z[k][1] + I[4] * z[k][2];
            Iz[k][1] = I[3] * z[k][0] + I[1] * z[k][1] + I[5] * z[k][2];
            Iz[k][2] = I[4] * z[k][0] + I[5] * z[k][1] + I[2] * z[k][2];
        }
#pragma unroll
        for (int j = 0; j <= i; ++j)
#pragma unroll
            for (int k = 0; k <= j; ++k) Mm[j][k] += m * dot3(jv[j], jv[k]) + dot3(z[j], Iz[k]);
    }
    R idg[NJ];
    chol_lower<NJ>(Mm, idg);
    R rhs[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) rhs[j] = tau[j] + tauext[j] - h[j];
    chol_solve<NJ>(Mm, idg, rhs);
#pragma unroll
    for (int j = 0; j < NJ; ++j) out.qdd[j] = rhs[j];

    if (FORCE) {
        // tau_F = v - g(q) (force_mode 0) or v; g(q) = sum_i J_v,i^T (-m_i g)
        R tF[NJ];
        if (Cst.force_mode == 0) {
            R fg[NJ][3], zero[NJ][3], gq[NJ];
#pragma unroll
            for (int i = 0; i < NJ; ++i)
#pragma unroll
                for (int c = 0; c < 3; ++c) { fg[i][c] = -Mdl.L[i].m * Mdl.g[c]; zero[i][c] = R(0); }
            jt_accumulate(z, p, cm, fg, zero, gq);
#pragma unroll
            for (int j = 0; j < NJ; ++j) tF[j] = v[j] - gq[j];
        } else {
#pragma unroll
            for (int j = 0; j < NJ; ++j) tF[j] = v[j];
        }
        // EE Jacobian rows [J_v; J_w] at the EE point
        R J[6][NJ];
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            R rj[3] = {out.pee[0] - p[j][0], out.pee[1] - p[j][1], out.pee[2] - p[j][2]}, jv[3];
            cross3(z[j], rj, jv);
            J[0][j] = jv[0]; J[1][j] = jv[1]; J[2][j] = jv[2];
            J[3][j] = z[j][0]; J[4][j] = z[j][1]; J[5][j] = z[j][2];
        }
        // with M = L L^T: A^T = L^-1 J^T (J M^-1 J^T = A A^T) and
        // y = L^-1 tau_F (J M^-1 tau_F = A y); the wrench is the
        // least-squares solution of A^T x = y (lsq_wrench)
        R At[NJ][6], y[NJ], b[6];
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                R s = J[r][i];
#pragma unroll
                for (int k = 0; k < i; ++k) s -= Mm[i][k] * At[k][r];
                At[i][r] = s * idg[i];
            }
            R s = tF[i];
#pragma unroll
            for (int k = 0; k < i; ++k) s -= Mm[i][k] * y[k];
            y[i] = s * idg[i];
        }
        lsq_wrench(At, y, b);
#pragma unroll
        for (int a = 0; a < 6; ++a) out.F[a] = b[a];
    }
}

}  // namespace mppi
