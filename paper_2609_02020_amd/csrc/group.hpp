// group.hpp -- one MPPI sample on a group of eight lanes: lane j holds
// joint j (j = 0..6) and lane 7 the end-effector frame.  The per-step work
// of Sec. III-A/B is spread over the group so that the chain of one
// sample's step is shorter than on one lane:
//
//   kinematics   every lane forms its joint transform Rp_j Rz(q_j), r_j
//                (lane 7: the fixed EE transform) and an inclusive scan of
//                transform compositions over the group gives every link
//                frame (R_j, p_j) at once, the EE pose in lane 7;
//   velocities   motion subspaces S_j = (z_j, (p_j - O) x z_j) in Pluecker
//                coordinates about one point O for all links (the step's
//                EE point, so that the distal links keep short moment
//                arms), where moving between links needs no transform, so
//                link twists are prefix sums
//                V_j = sum_{i<=j} S_i qd_i and velocity-product
//                accelerations prefix sums of V_i x S_i qd_i (gravity as
//                the base acceleration);
//   bias forces  f_j = I_j A_j + V_j x* I_j V_j (Newton-Euler per link,
//                lane 7 carries the negated wall wrench) and suffix sums
//                give h_j = S_j . sum_{i>=j} f_i, i.e. h(q, qd) of Eq. 5
//                less the external torque;
//   inertia      composite-rigid-body inertias Ic_j = sum_{i>=j} I_i
//                (suffix sums of the ten inertia parameters about O) give
//                the joint-space inertia M_ij = S_i . Ic_j S_j (i <= j),
//                the matrix of Eq. 8 plus the armature diagonal, row j in
//                lane j;
//   solve        the rows are gathered through the group's LDS area and
//                every lane factors M = L D L^T (no pivoting: M is SPD)
//                and solves Eq. 6 for the whole qdd; lane j keeps qdd_j;
//   force        (Eqs. 12-13) with J the EE Jacobian about the EE point
//                (columns (z_j, (p_j - p_ee) x z_j), short moment arms
//                where the estimate is taken) and M = L D L^T:
//                lane r (r < 6) solves L y = (row r of J)^T, lane 6
//                L y = tau_F, and D^-1/2 y is column j of [A^T | y'] with
//                J M^-1 J^T = A A^T and J M^-1 tau_F = A y'; the wrench is
//                the least-squares solution of A^T x = y' by modified
//                Gram-Schmidt with column j in lane j (six broadcast
//                steps) and a back substitution in every lane -- without
//                forming J M^-1 J^T, whose condition number (the square of
//                A's) exceeds 1 / u32 near kinematic singularities;
//   cost         lane 7 adds the pose and force terms of Eqs. 9-13, lanes
//                0..6 their joint's limit and torque terms (Eq. 14), and
//                the collision pairs of Eq. 15 are dealt over the eight
//                lanes; the group sums its lanes once, after the horizon.
//
// The code is written per lane against a group object G that provides the
// cross-lane moves (shr<D>: value of lane j - D, 0 for j < D; shr_one<D>:
// the same with 1 for j < D; add_shr<D> /
// add_shl<D>: x plus the value of lane j - D / j + D, plus 0 where there
// is none; bcast<K>: of lane K), sum (over the group), sync() (orders the
// group's LDS area) and shm (that area, kGxCount values).  On the device G
// is eight lanes of a row of 16, two groups interleaved (joint j in lane
// 2 j + p), so that DPP row shifts by 2 D stay within a group and fill the
// lanes without a source with 0, and a shift-and-add is one instruction; a
// host emulation runs the same code on eight threads in lockstep at every
// cross-lane move.
#pragma once

#include "rollout.hpp"

namespace mppi {

constexpr int kGroup = 8;
// group LDS area (values of the rollout type)
constexpr int kGxS = 16;                   // slot: S_j (6), 10 unused
constexpr int kGxSF = 0;                   // [8][kGxS]
constexpr int kGxRow = kGxSF + 8 * kGxS;   // [8][9]: M row j, tau - h, tau_F
constexpr int kGxOm = kGxRow + 8 * 9;      // [8][8]: the LDL^T factor of M (row i: L below the diagonal,
                                           // 1 / d_i on it), then lane j's column of the force solve's
                                           // triangular factor
constexpr int kGxH = kGxOm + 8 * 8;        // [8][12]: handoff to the cost part: q, qd, v, p_j, h_c, m_c
                                           // (lanes 0..6); lane 7: p_ee, R_ee
constexpr int kGxCount = kGxH + 8 * 12;    // 424

// Per-lane constants of the group rollout (lane 7: the EE frame, massless).
template <typename R> struct GroupLink {
    R Rp[9], rp[3];   // joint frame in the parent frame (lane 7: R_ee, r_ee)
    R Ic[6], com[3], m, arm;
    R qmin, qmax, qdmax, taumax, qrest;
    R sigma, sig_c;   // sampling scale of this joint (0 in lane 7)
    R live;           // 1 for a joint, 0 for lane 7
};

template <typename R> MPPI_HD void group_link(const ModelM<R>& M, const CostM<R>& C, int j, GroupLink<R>& G)
{
    const bool live = j < NJ;
    const LinkM<R>& L = M.L[live ? j : NJ - 1];
#pragma unroll
    for (int a = 0; a < 9; ++a) G.Rp[a] = live ? L.Rp[a] : M.Ree[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        G.rp[a] = live ? L.rp[a] : M.ree[a];
        G.com[a] = live ? L.com[a] : R(0);
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) G.Ic[a] = live ? L.Ic[a] : R(0);
    G.m = live ? L.m : R(0);
    G.arm = live ? L.arm : R(0);
    G.qmin = L.qmin; G.qmax = L.qmax; G.qdmax = L.qdmax; G.taumax = L.taumax;
    G.qrest = C.q_rest[live ? j : NJ - 1];
    G.sigma = live ? C.sigma[j] : R(0);
    G.sig_c = live ? C.sig_c[j] : R(0);
    G.live = live ? R(1) : R(0);
}

// This lane's normal of step t: Philox call j / 4 of the counter (c, t, k,
// tick), Box-Muller pair (j / 2) mod 2, cosine (even j) or sine branch --
// the same u32 words and the same arithmetic as normals8, one normal per lane.
template <typename R> MPPI_HD R group_normal(uint64_t seed, uint32_t tick, uint32_t k, uint32_t t, int j)
{
    uint32_t x0 = (uint32_t)(j >> 2), x1 = t, x2 = k, x3 = tick;
    philox10(x0, x1, x2, x3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const bool hi = (j >> 1) & 1;
    R z0, z1;
    box_muller_pair<R>(hi ? x2 : x0, hi ? x3 : x1, z0, z1);
    return (j & 1) ? z1 : z0;
}

// the perturbation recursion of noise_step for this lane's joint
template <typename R> MPPI_HD R group_noise_step(const CostM<R>& C, const GroupLink<R>& L, R z, R du, int t)
{
    return (t == 0 || C.rho == R(0)) ? L.sigma * z : C.rho * du + L.sig_c * z;
}

// ---------------------------------------------------------------------------
// scans over the group
// ---------------------------------------------------------------------------
// inclusive prefix composition of (Q, t) (child frame in the parent frame):
// (Qa, ta) o (Qb, tb) = (Qa Qb, Qa tb + ta), earlier joints on the left;
// lanes j < D compose with the identity (I, 0) that the shift leaves them
template <int D, typename R, class G> MPPI_HD void scan_frames(const G& g, R* Q, R* t)
{
    R Qp[9], tp[3];
#pragma unroll
    for (int a = 0; a < 9; ++a)
        Qp[a] = (a % 4 == 0) ? g.template shr_one<D>(Q[a]) : g.template shr<D>(Q[a]);
#pragma unroll
    for (int a = 0; a < 3; ++a) tp[a] = g.template shr<D>(t[a]);
    R nt[3];
    mv3(Qp, t, nt);
    t[0] = nt[0] + tp[0]; t[1] = nt[1] + tp[1]; t[2] = nt[2] + tp[2];
    mm3(Qp, Q, Q);
}
// Inclusive prefix and suffix sums over the group (Hillis-Steele: three
// shift-and-add rounds, lanes past the ends adding 0)
template <int N, typename R, class G> MPPI_HD void prefix_sum(const G& g, R* x)
{
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = g.template add_shr<1>(x[a]);
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = g.template add_shr<2>(x[a]);
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = g.template add_shr<4>(x[a]);
}
template <int N, typename R, class G> MPPI_HD void suffix_sum(const G& g, R* x)
{
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = g.template add_shl<1>(x[a]);
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = g.template add_shl<2>(x[a]);
#pragma unroll
    for (int a = 0; a < N; ++a) x[a] = g.template add_shl<4>(x[a]);
}

// EE pose of the group: lane j gets its link frame (lane 7: R_ee, p_ee)
template <typename R, class G> MPPI_HD void group_fk(const G& g, const GroupLink<R>& L, R q, R* Q, R* p)
{
    R c, s;
    sincos_(q, &s, &c);
    joint_rot(L.Rp, c, s, Q);
    p[0] = L.rp[0]; p[1] = L.rp[1]; p[2] = L.rp[2];
    scan_frames<1>(g, Q, p);
    scan_frames<2>(g, Q, p);
    scan_frames<4>(g, Q, p);
}

// The cost weights that the group's running and terminal costs read at
// every step, held in registers: read once with the other reads of a
// step, where reads from the cost copy in LDS inside the EE lane's branch
// would each wait for their own round trip.
template <typename R> struct GroupCostW {
    R W_pos[3], W_ori[3], W_force[6], W_reg[6];
    R w_q, w_qd, w_post, w_tau;
    int has_ori;
};
template <typename R> MPPI_HD void group_cost_w(const CostM<R>& C, GroupCostW<R>& w)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) { w.W_pos[a] = C.W_pos[a]; w.W_ori[a] = C.W_ori[a]; }
#pragma unroll
    for (int a = 0; a < 6; ++a) { w.W_force[a] = C.W_force[a]; w.W_reg[a] = C.W_reg[a]; }
    w.w_q = C.w_q; w.w_qd = C.w_qd; w.w_post = C.w_post; w.w_tau = C.w_tau;
    w.has_ori = C.has_ori;
}

// pose terms of Eqs. 9-11 from the EE frame (R_ee = R_n R_ee,fixed)
template <typename R> MPPI_HD R pose_cost(const GroupCostW<R>& W, const TargetM<R>& tg, const R* pee, const R* Re)
{
    R s = W.W_pos[0] * sq(tg.p_des[0] - pee[0]) + W.W_pos[1] * sq(tg.p_des[1] - pee[1]) +
          W.W_pos[2] * sq(tg.p_des[2] - pee[2]);
    if (W.has_ori) {
        R Rerr[9], rho[3];
        mm3(tg.RdT, Re, Rerr);
        so3_log(Rerr, rho);
        s += W.W_ori[0] * rho[0] * rho[0] + W.W_ori[1] * rho[1] * rho[1] + W.W_ori[2] * rho[2] * rho[2];
    }
    return s;
}
// this lane's joint-limit, velocity-limit and posture terms (Eq. 14 C_joint)
template <typename R> MPPI_HD R joint_cost1(const GroupCostW<R>& W, const GroupLink<R>& L, R q, R qd)
{
    return W.w_q * (sq(hinge(q - L.qmax)) + sq(hinge(L.qmin - q))) + W.w_qd * sq(hinge(abs_(qd) - L.qdmax)) +
           W.w_post * sq(q - L.qrest);
}
// force terms of Eq. 12 (the arithmetic of force_cost)
template <typename R> MPPI_HD R group_force_cost(const GroupCostW<R>& W, const TargetM<R>& tg, const R* F)
{
    R s = R(0);
#pragma unroll
    for (int a = 0; a < 6; ++a) s += W.W_force[a] * sq(tg.F_des[a] - F[a]) + W.W_reg[a] * F[a] * F[a];
    return s;
}

// One modified Gram-Schmidt step of lsq_wrench on the group: column S of
// [A^T | y] (lane S) is broadcast; every lane takes its entry of row S of
// the triangular factor, Rc[S] = q_S . col (q_S the normalised column S),
// and lanes j > S remove the q_S component from their column.  idg[S] =
// 1 / |column S| in every lane.
template <int S, typename R, class G> MPPI_HD void group_mgs_step(const G& g, R* col, R* Rc, R* idg)
{
    R u[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) u[i] = g.template bcast<S>(col[i]);
    R n2 = R(0), d = R(0);
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        n2 = fma_(u[i], u[i], n2);
        d = fma_(u[i], col[i], d);
    }
    const R r = rsqrt_sqrt_(n2);
    idg[S] = rcp_(r);
    Rc[S] = d * idg[S];
    const R coef = g.j > S ? d * idg[S] * idg[S] : R(0);
#pragma unroll
    for (int i = 0; i < NJ; ++i) col[i] = fma_(-coef, u[i], col[i]);
}

// What a group step leaves for inspection (host checks): lane 7's EE pose,
// the force estimate (FORCE) and this lane's qdd.
template <typename R> struct GroupStepOut {
    R qdd;
    R pee[3], Re[9];
    R F[6];
};

// M = L D L^T (unit lower L, lower triangle in Lm, 1/d in id) of the rows
// gathered in the group area, in every lane; b0 (may be null): the
// right-hand side tau - h of the rows.
template <typename R> struct GroupFactor {
    R Lm[NJ][NJ];
    R id[NJ];
};
template <typename R> MPPI_HD void group_factor(const R* X, GroupFactor<R>& f, R* b0)
{
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
#pragma unroll
        for (int c = 0; c <= i; ++c) f.Lm[i][c] = X[kGxRow + i * 9 + c];
        if (b0) b0[i] = X[kGxRow + i * 9 + 7];
    }
#pragma unroll
    for (int k = 0; k < NJ; ++k) {
        f.id[k] = rcp_(f.Lm[k][k]);
        R u[NJ];
#pragma unroll
        for (int i = k + 1; i < NJ; ++i) { u[i] = f.Lm[i][k]; f.Lm[i][k] = u[i] * f.id[k]; }
#pragma unroll
        for (int i = k + 1; i < NJ; ++i)
#pragma unroll
            for (int c = k + 1; c <= i; ++c) f.Lm[i][c] = fma_(-f.Lm[i][k], u[c], f.Lm[i][c]);
    }
}

// Dynamics part of one step (Eqs. 5-6): kinematics, twists, bias forces,
// composite inertias, the rows of M and their right-hand sides in the group
// area X, the factorisation (into *fac when given) and qdd.  Returns this
// lane's qdd (0 in lane 7); p, Q receive this lane's frame (lane 7: the EE
// pose).  tau: this lane's joint torque (sampled torque plus any
// joint-space external torque); v: the sampled torque (tau_F).
// FDYN: the input of the force estimate that the rows do not hold (tau_F
// in column 8 of the rows) is formed here, on the
// dynamics chain; otherwise group_cost forms it from the handoff.  The
// update kernel chooses FDYN when the cost part also carries the collision
// pairs, so that neither part runs both.
template <typename R, bool FORCE, class G, bool FDYN = false, bool HANDOFF = false>
MPPI_HD R group_dynamics(const G& g, const GroupLink<R>& L, const CostM<R>& C, const R* grav, int ext, R q, R qd,
                         R tau, R v, R* X, GroupFactor<R>* fac, R* p, R* Q)
{
    const int j = g.j;
    const bool ee = j == kGroup - 1;
    // the wall's constants, read ahead of the chain that uses them
    R wn[3], wd0 = R(0), wk = R(0), wc = R(0);
    if (ext == EXTW_WALL) {
#pragma unroll
        for (int a = 0; a < 3; ++a) wn[a] = C.wall_n[a];
        wd0 = C.wall_d0;
        wk = C.wall_k;
        wc = C.wall_c;
    }
    sched_fence();

    // ---- kinematics: link frames (lane 7: the EE frame)
    group_fk(g, L, q, Q, p);
    // spatial quantities are taken about the EE point O = p_ee of this
    // step (a fixed point in space for the step): the moment arms of the
    // distal links, whose small inertias set the small entries of M, stay
    // at link length, where arms about the world origin would be the reach
    const R pe[3] = {g.template bcast<kGroup - 1>(p[0]), g.template bcast<kGroup - 1>(p[1]),
                     g.template bcast<kGroup - 1>(p[2])};
    const R pr[3] = {p[0] - pe[0], p[1] - pe[1], p[2] - pe[2]};
    // motion subspace about O (lane 7: none); its linear part (p_j - p_ee)
    // x z_j is also the EE Jacobian's linear column about the EE point
    R z[3] = {Q[2] * L.live, Q[5] * L.live, Q[8] * L.live}, pz[3];
    cross3(pr, z, pz);
    // link inertia about O: mass m, first moment h = m c, rotational I_O
    R cw[3], Ib[6];
    mv3(Q, L.com, cw);
    cw[0] += pr[0]; cw[1] += pr[1]; cw[2] += pr[2];
    congr_sym3<false>(Q, L.Ic, Ib);
    R In[10];   // h[3], m, I_O[6]
    In[0] = L.m * cw[0]; In[1] = L.m * cw[1]; In[2] = L.m * cw[2]; In[3] = L.m;
    {
        const R c00 = cw[0] * cw[0], c11 = cw[1] * cw[1], c22 = cw[2] * cw[2];
        In[4] = Ib[0] + L.m * (c11 + c22);
        In[5] = Ib[1] + L.m * (c00 + c22);
        In[6] = Ib[2] + L.m * (c00 + c11);
        In[7] = Ib[3] - In[0] * cw[1];
        In[8] = Ib[4] - In[0] * cw[2];
        In[9] = Ib[5] - In[1] * cw[2];
    }

    // ---- twists V_j = sum_{i<=j} S_i qd_i
    R Sq[6] = {z[0] * qd, z[1] * qd, z[2] * qd, pz[0] * qd, pz[1] * qd, pz[2] * qd};
    R V[6] = {Sq[0], Sq[1], Sq[2], Sq[3], Sq[4], Sq[5]};
    prefix_sum<6>(g, V);
    // velocity-product accelerations V_j x (S_j qd_j), prefix-summed, plus
    // the base acceleration -g
    R A[6];
    {
        R t1[3], t2[3], t3[3];
        cross3(V, Sq, t1);
        cross3(V, Sq + 3, t2);
        cross3(V + 3, Sq, t3);
        A[0] = t1[0]; A[1] = t1[1]; A[2] = t1[2];
        A[3] = t2[0] + t3[0]; A[4] = t2[1] + t3[1]; A[5] = t2[2] + t3[2];
    }
    prefix_sum<6>(g, A);
    A[3] -= grav[0]; A[4] -= grav[1]; A[5] -= grav[2];

    // ---- link forces f = I A + V x* (I V)
    auto inertia_mul = [&](const R* P, const R* x, R* y) {
        // (I_O w + h x v, m v - h x w)
        R hv[3], hw[3];
        cross3(P, x + 3, hv);
        cross3(P, x, hw);
        y[0] = P[4] * x[0] + P[7] * x[1] + P[8] * x[2] + hv[0];
        y[1] = P[7] * x[0] + P[5] * x[1] + P[9] * x[2] + hv[1];
        y[2] = P[8] * x[0] + P[9] * x[1] + P[6] * x[2] + hv[2];
        y[3] = P[3] * x[3] - hw[0];
        y[4] = P[3] * x[4] - hw[1];
        y[5] = P[3] * x[5] - hw[2];
    };
    R f[6];
    {
        R IV[6], t1[3], t2[3], t3[3];
        inertia_mul(In, A, f);
        inertia_mul(In, V, IV);
        cross3(V, IV, t1);
        cross3(V + 3, IV + 3, t2);
        cross3(V, IV + 3, t3);
        f[0] += t1[0] + t2[0]; f[1] += t1[1] + t2[1]; f[2] += t1[2] + t2[2];
        f[3] += t3[0]; f[4] += t3[1]; f[5] += t3[2];
    }
    if (ext == EXTW_WALL) {
        // unilateral spring-damper at the EE point (lane 7's frame origin,
        // the reference point O: the EE point velocity is V's linear part
        // and the wall force has no moment about O)
        const R delta = wd0 - dot3(wn, p);
        const R ddelta = -dot3(wn, V + 3);
        const R mag = hinge(wk * delta + wc * ddelta);
        if (ee) {
            f[3] -= wn[0] * mag; f[4] -= wn[1] * mag; f[5] -= wn[2] * mag;
        }
    }

    // ---- subtree sums: bias forces and composite inertias
    suffix_sum<6>(g, f);
    suffix_sum<10>(g, In);
    const R hq = dot3(z, f) + dot3(pz, f + 3);
    // Ic S and the gravity torque S . Ic (0, -g)
    R Fm[6];
    {
        R Sv[6] = {z[0], z[1], z[2], pz[0], pz[1], pz[2]};
        inertia_mul(In, Sv, Fm);
    }

    // ---- gather S (Ic S stays in this lane)
    R* slot = X + kGxSF + j * kGxS;
#pragma unroll
    for (int a = 0; a < 3; ++a) { slot[a] = z[a]; slot[3 + a] = pz[a]; }
    if (FORCE && FDYN) {
        // tau_F (less the gravity torque S . Ic (0, -g) when force_mode is 0)
        R tf = v;
        if (C.force_mode == 0) {
            const R ag[3] = {-grav[0], -grav[1], -grav[2]};
            R ha[3];
            cross3(In, ag, ha);
            tf = v - (dot3(z, ha) + In[3] * dot3(pz, ag));
        }
        X[kGxRow + j * 9 + 8] = ee ? R(0) : tf;
    }
    g.sync();
    // row j of M up to the diagonal: M_jc = S_c . (Ic S)_j (c <= j), plus
    // the armature; every lane reads the slots at the same offsets and
    // multiplies by its own Ic S.  Above the diagonal the same products
    // are not M (nothing reads that part of the rows).
    R Sc[NJ][6], row[NJ];
#pragma unroll
    for (int c = 0; c < NJ; ++c)
#pragma unroll
        for (int a = 0; a < 6; ++a) Sc[c][a] = X[kGxSF + c * kGxS + a];
    sched_fence();   // the 42 reads in one round trip
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
        const R* S = Sc[c];
        R s = S[0] * Fm[0] + S[1] * Fm[1] + S[2] * Fm[2] + S[3] * Fm[3] + S[4] * Fm[4] + S[5] * Fm[5];
        row[c] = s + (c == j ? L.arm : R(0));
    }
    // the EE lane's slot holds no motion subspace: its rows are 0
    if (ee) {
#pragma unroll
        for (int c = 0; c < NJ; ++c) row[c] = R(0);
    }
#pragma unroll
    for (int c = 0; c < NJ; ++c) X[kGxRow + j * 9 + c] = row[c];
    X[kGxRow + j * 9 + 7] = tau - hq;
    g.sync();

    // ---- Eq. 6: qdd = L^-T D^-1 L^-1 (tau + tau_ext - h)
    GroupFactor<R> local;
    GroupFactor<R>& F = fac ? *fac : local;
    R b0[NJ], x[NJ];
    group_factor(X, F, b0);
    // handoff to the cost part: pre-step q, qd, v, the joint origin and the
    // subtree's mass and first moment (lanes 0..6), the EE pose (lane 7);
    // written once the rows are read, so that the row reads do not queue
    // behind these writes
    R* h = X + kGxH + j * 12;
    if (ee) {
#pragma unroll
        for (int a = 0; a < 3; ++a) h[a] = p[a];
#pragma unroll
        for (int a = 0; a < 9; ++a) h[3 + a] = Q[a];
    } else {
        h[0] = q; h[1] = qd; h[2] = v;
        h[3] = p[0]; h[4] = p[1]; h[5] = p[2];
        if (FORCE && !FDYN) { h[6] = In[0]; h[7] = In[1]; h[8] = In[2]; h[9] = In[3]; }
    }
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        R s = b0[i];
#pragma unroll
        for (int c = 0; c < i; ++c) s = fma_(-F.Lm[i][c], x[c], s);
        x[i] = s;
    }
#pragma unroll
    for (int i = NJ - 1; i >= 0; --i) {
        R s = x[i] * F.id[i];
#pragma unroll
        for (int c = i + 1; c < NJ; ++c) s = fma_(-F.Lm[c][i], x[c], s);
        x[i] = s;
    }
    if (FORCE && HANDOFF && j == 0) {
        // for the cost part (HANDOFF): row i of L below the diagonal and
        // 1 / d_i on it, in the kGxOm rows, so that it does not factorise
        // M again (one lane writes; the other lanes have read M)
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
#pragma unroll
            for (int c = 0; c < i; ++c) X[kGxOm + i * 8 + c] = F.Lm[i][c];
            X[kGxOm + i * 8 + i] = F.id[i];
        }
    }
    R qj = R(0);
#pragma unroll
    for (int i = 0; i < NJ; ++i) qj = (i == j) ? x[i] : qj;
    return qj;
}

// Cost part of one step: the force estimate of Eq. 13 (FORCE) from the
// factor of M (fac; when null, the one group_dynamics left in X with
// HANDOFF, else M's rows in X factorised again) and the Jacobian rows left
// in X, and this lane's running cost at (x_t, v_t): pose and
// force terms in lane 7 (pee, Re: its EE pose), joint-limit and torque
// terms in lanes 0..6, and with COLL the collision term of Eqs. 14-15 with
// the pairs dealt over the lanes (pair i to lane i mod 8; link segments
// from the joint origins and the EE point in the handoff).  Uses the kGxOm
// part of X.
template <typename R, bool FORCE, bool COLL, class G, bool FDYN = false, bool HANDOFF = false>
MPPI_HD R group_cost(const G& g, const GroupLink<R>& L, const CostM<R>& C, const TargetM<R>& tg, const R* grav,
                     R* X, const GroupFactor<R>* fac, R q, R qd, R v, const R* pee, const R* Re,
                     R* Fout = nullptr)
{
    const int j = g.j;
    const bool ee = j == kGroup - 1;
    GroupCostW<R> W;
    group_cost_w(C, W);
    R sj[6];   // this lane's motion subspace (the gravity torque of tau_F)
#pragma unroll
    for (int a = 0; a < 6; ++a) sj[a] = X[kGxSF + j * kGxS + a];
    sched_fence();   // with the handoff reads: one round trip
    R ell = R(0);
    if (COLL) {
        // segment id s: link s from P[s] to P[s + 1] (P[7] = EE point), or
        // obstacle s - 7
        auto ends = [&](int sid, R* e0, R* e1) {
            if (sid < NJ) {
                const R* a = X + kGxH + sid * 12 + 3;
                const R* b = X + kGxH + (sid + 1) * 12 + (sid + 1 < NJ ? 3 : 0);
#pragma unroll
                for (int c = 0; c < 3; ++c) { e0[c] = a[c]; e1[c] = b[c]; }
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) { e0[c] = C.obs[sid - NJ][c]; e1[c] = C.obs[sid - NJ][3 + c]; }
            }
        };
        R hits = R(0);
        g.sync();   // the other lanes' handoff (written at the end of the dynamics part)
        for (int i = j; i < C.n_pairs; i += kGroup) {
            R a0[3], a1[3], b0[3], b1[3];
            ends(C.pa[i], a0, a1);
            ends(C.pb[i], b0, b1);
            if (seg_dist2(a0, a1, b0, b1) < C.dth2[i]) hits += R(1);
        }
        ell += C.w_coll * hits;
    }
    if (FORCE) {
        // tau_F of this lane's joint: v, less the gravity torque
        // S . Ic (0, -g) of the subtree when force_mode is 0
        if (!FDYN) {
            // the gravity torque is formed whatever force_mode says, so that
            // its reads join the step's first batch instead of a branch
            const R* hj = X + kGxH + j * 12;
            const R ag[3] = {-grav[0], -grav[1], -grav[2]};
            R ha[3];
            cross3(hj + 6, ag, ha);
            const R tg0 = v - (dot3(sj, ha) + hj[9] * dot3(sj + 3, ag));
            const R tf = C.force_mode == 0 ? tg0 : v;
            X[kGxRow + j * 9 + 8] = ee ? R(0) : tf;
        }
        // row r of the EE Jacobian about p_ee at joint i: z_i (r < 3), then
        // (p_i - p_ee) x z_i, i.e. component r of the motion subspace S_i
        // about the EE point
        const int r = j < 6 ? j : 5;
        R Jr[NJ];
#pragma unroll
        for (int i = 0; i < NJ; ++i) Jr[i] = X[kGxSF + i * kGxS + r];
        g.sync();
        GroupFactor<R> local;
        if (!fac && HANDOFF) {
            // the factor that group_dynamics left in the kGxOm rows
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
#pragma unroll
                for (int c = 0; c < i; ++c) local.Lm[i][c] = X[kGxOm + i * 8 + c];
                local.id[i] = X[kGxOm + i * 8 + i];
            }
        } else if (!fac) {
            group_factor(X, local, (R*)nullptr);
        }
        const GroupFactor<R>& Fc = fac ? *fac : local;
        R bF[NJ];
#pragma unroll
        for (int i = 0; i < NJ; ++i) bF[i] = X[kGxRow + i * 9 + 8];
        // ---- lane r < 6 solves for row r of J, lane 6 (and 7) for tau_F;
        // scaled by D^-1/2 that is column j of [A^T | y] with Omega = A A^T
        // and J M^-1 tau_F = A y (M = L D L^T, A^T = D^-1/2 L^-1 J^T)
        R col[NJ];
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
            R s = j < 6 ? Jr[i] : bF[i];
#pragma unroll
            for (int c = 0; c < i; ++c) s = fma_(-Fc.Lm[i][c], col[c], s);
            col[i] = s;
        }
#pragma unroll
        for (int i = 0; i < NJ; ++i) col[i] *= rsqrt_sqrt_(Fc.id[i]);
        // least squares A^T x = y by modified Gram-Schmidt over the lanes
        // (lsq_wrench's arithmetic with column j in lane j): this lane's
        // column of the triangular factor (Rc[s], s < j; lane 6: Q^T y)
        R Rc[6], idg[6];
        group_mgs_step<0>(g, col, Rc, idg);
        group_mgs_step<1>(g, col, Rc, idg);
        group_mgs_step<2>(g, col, Rc, idg);
        group_mgs_step<3>(g, col, Rc, idg);
        group_mgs_step<4>(g, col, Rc, idg);
        group_mgs_step<5>(g, col, Rc, idg);
#pragma unroll
        for (int s = 0; s < 6; ++s) X[kGxOm + j * 8 + s] = Rc[s];
        g.sync();
        // x = Rm^-1 Q^T y in every lane: (moment, force) about p_ee; the
        // triangle and Q^T y are read in one round trip
        R Rm[6][6], qy[6], bb[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            qy[s] = X[kGxOm + 6 * 8 + s];
#pragma unroll
            for (int c = s + 1; c < 6; ++c) Rm[c][s] = X[kGxOm + c * 8 + s];
        }
        sched_fence();
#pragma unroll
        for (int s = 5; s >= 0; --s) {
            R t = qy[s];
#pragma unroll
            for (int c = s + 1; c < 6; ++c) t = fma_(-Rm[c][s], bb[c], t);
            bb[s] = t * idg[s];
        }
        const R F[6] = {bb[3], bb[4], bb[5], bb[0], bb[1], bb[2]};
        if (ee) ell += group_force_cost(W, tg, F);
        if (Fout) {
#pragma unroll
            for (int a = 0; a < 6; ++a) Fout[a] = F[a];
        }
    }
    if (ee) ell += pose_cost(W, tg, pee, Re);
    else ell += joint_cost1(W, L, q, qd) + W.w_tau * sq(hinge(abs_(v) - L.taumax));
    return ell;
}

// One step of Eqs. 5-7 and the running cost at the pre-step state (x_t,
// v_t) on one group of lanes: returns this lane's share of l_t and sets
// qdd (0 in lane 7).
template <typename R, bool FORCE, class G, bool COLL = false>
MPPI_HD R group_step(const G& g, const GroupLink<R>& L, const CostM<R>& C, const TargetM<R>& tg, const R* grav,
                     int ext, R q, R qd, R tau, R v, R& qdd, GroupStepOut<R>* dbg = nullptr)
{
    GroupFactor<R> fac;
    R p[3], Q[9], F[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    qdd = group_dynamics<R, FORCE, G, COLL>(g, L, C, grav, ext, q, qd, tau, v, g.shm, &fac, p, Q);
    const R ell = group_cost<R, FORCE, COLL, G, COLL>(g, L, C, tg, grav, g.shm, &fac, q, qd, v, p, Q, F);
    if (dbg) {
        dbg->qdd = qdd;
#pragma unroll
        for (int a = 0; a < 3; ++a) dbg->pee[a] = p[a];
#pragma unroll
        for (int a = 0; a < 9; ++a) dbg->Re[a] = Q[a];
#pragma unroll
        for (int a = 0; a < 6; ++a) dbg->F[a] = F[a];
    }
    return ell;
}

// Terminal cost phi(x_T) = w_T (C_pos + C_ori + C_joint)(x_T): this lane's share.
template <typename R, class G>
MPPI_HD R group_terminal(const G& g, const GroupLink<R>& L, const CostM<R>& C, const TargetM<R>& tg, R q, R qd)
{
    GroupCostW<R> W;
    group_cost_w(C, W);
    R Q[9], p[3];
    group_fk(g, L, q, Q, p);
    const R s = g.j == kGroup - 1 ? pose_cost(W, tg, p, Q) : joint_cost1(W, L, q, qd);
    return C.w_T * s;
}

// One sample's rollout on the group (Eq. 3 with the dynamics of Sec. III-A):
// returns the sample's total cost S_k in every lane.  Us: [T][7] nominal
// torques; te: this lane's joint-space external torque (constant mode);
// noise_out, noise_lds (either may be null): du[t][j] of this lane's joint
// at (7 t + j) * stride (lanes 0..6).  split: each step as its dynamics
// part and then its cost part (group_dynamics, group_cost with the factor
// of M handed over in the group area) instead of group_step.
template <typename R, bool FORCE, class G, typename UT, bool COLL = false>
MPPI_HD R group_rollout(const G& g, const GroupLink<R>& L, const CostM<R>& C, const TargetM<R>& tg,
                        const R* grav, R q, R qd, R te, const UT* Us, int T, uint64_t seed, uint32_t tick,
                        uint32_t k, R* noise_out, size_t noise_stride, R* noise_lds = nullptr, int lds_stride = 0,
                        bool split = false)
{
    const int j = g.j;
    const int jc = j < NJ ? j : NJ - 1;
    const int ext = C.ext_mode == EXTW_WALL ? EXTW_WALL : EXTW_NONE;
    const R dt = C.dt;
    R du = R(0), S = R(0);
    for (int t = 0; t < T; ++t) {
        const R z = group_normal<R>(seed, tick, k, (uint32_t)t, j);
        du = group_noise_step(C, L, z, du, t);
        if (noise_out && j < NJ) noise_out[(size_t)(t * NJ + j) * noise_stride] = du;
        if (noise_lds && j < NJ) noise_lds[(t * NJ + j) * lds_stride] = du;
        const R v = (R(Us[t * NJ + jc]) + du) * L.live;
        R qdd;
        if (split) {
            // the dynamics and cost parts in sequence, the factor of M
            // handed over through the group area instead of held in
            // registers across the cost part
            R p[3], Q[9];
            qdd = group_dynamics<R, FORCE, G, COLL, true>(g, L, C, grav, ext, q, qd, v + te, v, g.shm, nullptr, p, Q);
            S += group_cost<R, FORCE, COLL, G, COLL, true>(g, L, C, tg, grav, g.shm, nullptr, q, qd, v, p, Q);
        } else {
            S += group_step<R, FORCE, G, COLL>(g, L, C, tg, grav, ext, q, qd, v + te, v, qdd);
        }
        qd += qdd * dt;
        q += qd * dt;
    }
    S += group_terminal(g, L, C, tg, q, qd);
    return g.sum(S);
}

}  // namespace mppi
