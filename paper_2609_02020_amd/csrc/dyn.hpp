// dyn.hpp -- per-sample rigid-body dynamics, noise and cost for the MPPI
// rollout kernels (gfx950).  Header-only, templated on the scalar type
// (float for the FP32 rollouts, double for FP64).
//
// What one rollout step computes (Sec. III-A/B of Im et al., "Real-Time
// Dynamics-Based Torque-Sampling MPPI ..."):
//   * forward kinematics of the 7-joint chain -> EE pose (Eq. 11 inputs);
//   * forward dynamics qdd = M^-1 (tau + tau_ext - h) (Eqs. 5-6), evaluated
//     without forming M by the articulated-body algorithm (Featherstone),
//     in link-local spatial coordinates [angular; linear];
//   * when the force cost is on, the EE wrench estimate of Eq. 13,
//     F_ee = Lambda J M^-1 tau_F, from two extra quantities that reuse the
//     articulated-body factors (U_i, D_i) of the same step:
//       - Omega_n = J_n M^-1 J_n^T, the inverse articulated inertia seen at
//         the last link, by the outward recursion
//           Omega_i = P_i X_i Omega_{i-1} X_i^T P_i^T + S D_i^-1 S^T,
//           P_i = 1 - S D_i^-1 U_i^T,   Omega_{-1} = 0 (fixed base);
//       - J_n M^-1 tau_F from one extra zero-velocity solve;
//     then x = Omega_n^-1 (J_n M^-1 tau_F) by a 6x6 Cholesky and
//     F_ee = T^-T x (T: last-link origin -> EE point, world axes).
//   * the running cost of Eqs. 9-14 and the semi-implicit Euler step of
//     Eq. 7 are applied by the caller.
//
// Layout: every joint is revolute about its local z (S = e_2).  Frame i in
// frame i-1: orientation Q_i = Rp_i Rz(q_i), origin rp_i.  Motion transform
// parent->child X_i = [E 0; -E rx E] with E = Q_i^T.  A symmetric 6x6 block
// matrix is stored as Sym6 {A (3x3 sym), B (3x3), C (3x3 sym)} =
// [A B; B^T C].
#pragma once

#include <cmath>
#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define MPPI_HD __host__ __device__ __forceinline__
#else
#define MPPI_HD inline
#endif

namespace mppi {

constexpr int NJ = 7;

// ---------------------------------------------------------------------------
// scalar math: device builtins on the GPU, libm on the host
// ---------------------------------------------------------------------------
MPPI_HD void sincos_(float x, float* s, float* c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    sincosf(x, s, c);
#else
    *s = std::sin(x); *c = std::cos(x);
#endif
}
MPPI_HD void sincos_(double x, double* s, double* c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    sincos(x, s, c);
#else
    *s = std::sin(x); *c = std::cos(x);
#endif
}
MPPI_HD void sincospi_(float x, float* s, float* c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    sincospif(x, s, c);
#else
    *s = std::sin(3.14159265358979323846 * x); *c = std::cos(3.14159265358979323846 * x);
#endif
}
MPPI_HD void sincospi_(double x, double* s, double* c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    sincospi(x, s, c);
#else
    *s = std::sin(3.14159265358979323846 * x); *c = std::cos(3.14159265358979323846 * x);
#endif
}
MPPI_HD float sqrt_(float x) { return std::sqrt(x); }
MPPI_HD double sqrt_(double x) { return std::sqrt(x); }
MPPI_HD float log_(float x) { return std::log(x); }
MPPI_HD double log_(double x) { return std::log(x); }
MPPI_HD float atan2_(float y, float x) { return std::atan2(y, x); }
MPPI_HD double atan2_(double y, double x) { return std::atan2(y, x); }
MPPI_HD float abs_(float x) { return std::fabs(x); }
MPPI_HD double abs_(double x) { return std::fabs(x); }

template <typename R> MPPI_HD R hinge(R x) { return x > R(0) ? x : R(0); }
template <typename R> MPPI_HD R sq(R x) { return x * x; }

// ---------------------------------------------------------------------------
// model and cost as the kernels read them
// ---------------------------------------------------------------------------
template <typename R> struct LinkM {
    R Rp[9];      // R_parent, row-major
    R rp[3];      // r_parent
    R Io[6];      // rotational inertia about the link-frame origin (xx yy zz xy xz yz)
    R mc[3];      // mass * CoM
    R m;          // mass
    R arm;        // armature
    R qmin, qmax, qdmax, taumax;
};

template <typename R> struct ModelM {
    LinkM<R> L[NJ];
    R Ree[9];     // EE frame in the last link frame
    R ree[3];     // EE point in the last link frame
    R g[3];       // world gravity
};

enum { EXTW_NONE = 0, EXTW_CONST = 1, EXTW_WALL = 2 };

template <typename R> struct CostM {
    R dt;
    R sigma[NJ];
    R W_pos[3], W_ori[3], W_force[6], W_reg[6];
    R w_q, w_qd, w_tau, w_post;
    R q_rest[NJ];
    R w_T;
    R F_ext[6];
    R wall_n[3];
    R wall_d0, wall_k, wall_c;
    int ext_mode;     // mppi_ext_mode
    int force_mode;   // 0: tau_F = v - g(q); 1: tau_F = v
    int has_ori;      // any W_ori != 0
    int has_force;    // any W_force / W_reg != 0
};

// ---------------------------------------------------------------------------
// 3-vector / 3x3 helpers
// ---------------------------------------------------------------------------
MPPI_HD constexpr int si(int i, int j) { return i == j ? i : i + j + 2; } // sym3 index

template <typename R> MPPI_HD void cross3(const R* a, const R* b, R* c)
{
    R x = a[1] * b[2] - a[2] * b[1];
    R y = a[2] * b[0] - a[0] * b[2];
    R z = a[0] * b[1] - a[1] * b[0];
    c[0] = x; c[1] = y; c[2] = z;
}
template <typename R> MPPI_HD R dot3(const R* a, const R* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
// y = Q x
template <typename R> MPPI_HD void mv3(const R* Q, const R* x, R* y)
{
    R t0 = Q[0] * x[0] + Q[1] * x[1] + Q[2] * x[2];
    R t1 = Q[3] * x[0] + Q[4] * x[1] + Q[5] * x[2];
    R t2 = Q[6] * x[0] + Q[7] * x[1] + Q[8] * x[2];
    y[0] = t0; y[1] = t1; y[2] = t2;
}
// y = Q^T x
template <typename R> MPPI_HD void mtv3(const R* Q, const R* x, R* y)
{
    R t0 = Q[0] * x[0] + Q[3] * x[1] + Q[6] * x[2];
    R t1 = Q[1] * x[0] + Q[4] * x[1] + Q[7] * x[2];
    R t2 = Q[2] * x[0] + Q[5] * x[1] + Q[8] * x[2];
    y[0] = t0; y[1] = t1; y[2] = t2;
}
// C = A B
template <typename R> MPPI_HD void mm3(const R* A, const R* B, R* C)
{
    R T[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            T[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
#pragma unroll
    for (int i = 0; i < 9; ++i) C[i] = T[i];
}
// Q = Rp Rz(q) from (cos q, sin q)
template <typename R> MPPI_HD void joint_rot(const R* Rp, R c, R s, R* Q)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R x = Rp[a * 3], y = Rp[a * 3 + 1];
        Q[a * 3] = c * x + s * y;
        Q[a * 3 + 1] = c * y - s * x;
        Q[a * 3 + 2] = Rp[a * 3 + 2];
    }
}

// out = Q M Q^T (TRANS = false) or Q^T M Q (TRANS = true), M symmetric
template <bool TRANS, typename R> MPPI_HD void congr_sym3(const R* Q, const R* M, R* out)
{
    auto q = [&](int i, int j) -> R { return TRANS ? Q[j * 3 + i] : Q[i * 3 + j]; };
    R T[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            T[i * 3 + j] = q(i, 0) * M[si(0, j)] + q(i, 1) * M[si(1, j)] + q(i, 2) * M[si(2, j)];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            out[si(i, j)] = T[i * 3] * q(j, 0) + T[i * 3 + 1] * q(j, 1) + T[i * 3 + 2] * q(j, 2);
}
// out = Q B Q^T (TRANS = false) or Q^T B Q (TRANS = true), B general
template <bool TRANS, typename R> MPPI_HD void congr_gen3(const R* Q, const R* B, R* out)
{
    auto q = [&](int i, int j) -> R { return TRANS ? Q[j * 3 + i] : Q[i * 3 + j]; };
    R T[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            T[i * 3 + j] = q(i, 0) * B[j] + q(i, 1) * B[3 + j] + q(i, 2) * B[6 + j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            out[i * 3 + j] = T[i * 3] * q(j, 0) + T[i * 3 + 1] * q(j, 1) + T[i * 3 + 2] * q(j, 2);
}

// (r x) M for general M, returned row-major: row i = r x (column) ...
// P_ij = sum_k rx_ik M_kj with rx = [[0,-r2,r1],[r2,0,-r0],[-r1,r0,0]]
template <typename R> MPPI_HD void rx_mul(const R* r, const R* M, R* P)
{
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        R m0 = M[j], m1 = M[3 + j], m2 = M[6 + j];
        P[j] = r[1] * m2 - r[2] * m1;
        P[3 + j] = r[2] * m0 - r[0] * m2;
        P[6 + j] = r[0] * m1 - r[1] * m0;
    }
}
// symmetric M (sym3 storage) -> full
template <typename R> MPPI_HD void sym_full(const R* S, R* F)
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) F[i * 3 + j] = S[si(i, j)];
}

template <typename R> struct Sym6 {
    R A[6];
    R B[9];
    R C[6];
};

// Force-side congruence child -> parent: out = X^T Ia X (Ia in child
// coordinates) for X = [E 0; -E rx E], E = Q^T.
// Rotate to parent axes: A1 = Q A Q^T, B1 = Q B Q^T, C1 = Q C Q^T; shift
// the reference point by r: C' = C1, B' = B1 + rx C1,
// A' = A1 + rx B1^T + (rx B1^T)^T - rx C1 rx.
template <typename R> MPPI_HD void congr_force(const R* Q, const R* r, const Sym6<R>& Ia, Sym6<R>& out)
{
    R A1[6], B1[9], C1[6], C1f[9], P[9], G[9], B1t[9];
    congr_sym3<false>(Q, Ia.A, A1);
    congr_gen3<false>(Q, Ia.B, B1);
    congr_sym3<false>(Q, Ia.C, C1);
    sym_full(C1, C1f);
    rx_mul(r, C1f, P);                       // P = rx C1
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) B1t[i * 3 + j] = B1[j * 3 + i];
    rx_mul(r, B1t, G);                       // G = rx B1^T
#pragma unroll
    for (int i = 0; i < 6; ++i) out.C[i] = C1[i];
#pragma unroll
    for (int i = 0; i < 9; ++i) out.B[i] = B1[i] + P[i];
    // (rx C1 rx)_ij = (P rx)_ij = P_i0 rx_0j + P_i1 rx_1j + P_i2 rx_2j with
    // rx = [[0, -r2, r1], [r2, 0, -r0], [-r1, r0, 0]]
    const R rx[9] = {R(0), -r[2], r[1], r[2], R(0), -r[0], -r[1], r[0], R(0)};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            R prx = P[i * 3] * rx[j] + P[i * 3 + 1] * rx[3 + j] + P[i * 3 + 2] * rx[6 + j];
            out.A[si(i, j)] = A1[si(i, j)] + G[i * 3 + j] + G[j * 3 + i] - prx;
        }
}

// Motion-side congruence parent -> child: out = X Om X^T (Om in parent
// coordinates).  Shift: A' = A, B' = A rx + B,
// C' = C - rx B - (rx B)^T - rx A rx; then rotate by E = Q^T.
template <typename R> MPPI_HD void congr_motion(const R* Q, const R* r, const Sym6<R>& Om, Sym6<R>& out)
{
    R Af[9], W[9], Bs[9], G[9], C2[6];
    sym_full(Om.A, Af);
    // W = A rx : W_ij = sum_k A_ik rx_kj  -> equals -(rx A)^T ... compute directly
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        R a0 = Af[i * 3], a1 = Af[i * 3 + 1], a2 = Af[i * 3 + 2];
        W[i * 3 + 0] = a1 * r[2] - a2 * r[1];
        W[i * 3 + 1] = a2 * r[0] - a0 * r[2];
        W[i * 3 + 2] = a0 * r[1] - a1 * r[0];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) Bs[i] = W[i] + Om.B[i];
    rx_mul(r, Om.B, G);                      // G = rx B
    // rx A rx = rx W
    R H[9];
    rx_mul(r, W, H);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            C2[si(i, j)] = Om.C[si(i, j)] - G[i * 3 + j] - G[j * 3 + i] - H[i * 3 + j];
    congr_sym3<true>(Q, Om.A, out.A);
    congr_gen3<true>(Q, Bs, out.B);
    congr_sym3<true>(Q, C2, out.C);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller
// ---------------------------------------------------------------------------
MPPI_HD void philox10(uint32_t& x0, uint32_t& x1, uint32_t& x2, uint32_t& x3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        x1 = (uint32_t)p1;
        x3 = (uint32_t)p0;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// 8 standard normals for counter (c, t, k, tick) c in {0, 1}, key = seed.
template <typename R> MPPI_HD void box_muller_pair(uint32_t xa, uint32_t xb, R& z0, R& z1)
{
    const R two_m32 = R(2.3283064365386962890625e-10);   // 2^-32
    R ua = (R(xa) + R(1)) * two_m32;                     // (0, 1]
    R ub = R(xb) * two_m32;                              // [0, 1)
    R rad = sqrt_(R(-2) * log_(ua));
    R s, c;
    sincospi_(R(2) * ub, &s, &c);
    z0 = rad * c;
    z1 = rad * s;
}

template <typename R> MPPI_HD void normals8(uint64_t seed, uint32_t tick, uint32_t k, uint32_t t, R* z)
{
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (uint32_t call = 0; call < 2; ++call) {
        uint32_t x0 = call, x1 = t, x2 = k, x3 = tick;
        philox10(x0, x1, x2, x3, k0, k1);
        box_muller_pair<R>(x0, x1, z[call * 4 + 0], z[call * 4 + 1]);
        box_muller_pair<R>(x2, x3, z[call * 4 + 2], z[call * 4 + 3]);
    }
}

// ---------------------------------------------------------------------------
// SO(3) log map (rotation vector), |rho| = theta in [0, pi]
// ---------------------------------------------------------------------------
template <typename R> MPPI_HD void so3_log(const R* M, R* rho)
{
    R vx = M[7] - M[5], vy = M[2] - M[6], vz = M[3] - M[1];
    R s = R(0.5) * sqrt_(vx * vx + vy * vy + vz * vz);
    R c = R(0.5) * (M[0] + M[4] + M[8] - R(1));
    R th = atan2_(s, c);
    const R tiny = sizeof(R) == 4 ? R(1e-4) : R(1e-7);
    if (s < tiny && c < R(0)) {
        // near pi: axis from the symmetric part (sign immaterial to the cost)
        R d0 = M[0] - c, d1 = M[4] - c, d2 = M[8] - c;
        R o01 = R(0.5) * (M[1] + M[3]), o02 = R(0.5) * (M[2] + M[6]), o12 = R(0.5) * (M[5] + M[7]);
        R a0, a1, a2, den;
        if (d0 >= d1 && d0 >= d2) { den = sqrt_(d0 * (R(1) - c)); a0 = d0 / den; a1 = o01 / den; a2 = o02 / den; }
        else if (d1 >= d2)        { den = sqrt_(d1 * (R(1) - c)); a0 = o01 / den; a1 = d1 / den; a2 = o12 / den; }
        else                      { den = sqrt_(d2 * (R(1) - c)); a0 = o02 / den; a1 = o12 / den; a2 = d2 / den; }
        if (a0 * vx + a1 * vy + a2 * vz < R(0)) { a0 = -a0; a1 = -a1; a2 = -a2; }
        rho[0] = th * a0; rho[1] = th * a1; rho[2] = th * a2;
        return;
    }
    R f = s > R(1e-12) ? R(0.5) * th / s : R(0.5);
    rho[0] = f * vx; rho[1] = f * vy; rho[2] = f * vz;
}

// 6x6 SPD solve (Cholesky), M given as Sym6, b overwritten by the solution.
template <typename R> MPPI_HD void chol6_solve(const Sym6<R>& S, R* b)
{
    R F[36];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            F[i * 6 + j] = S.A[si(i, j)];
            F[i * 6 + 3 + j] = S.B[i * 3 + j];
            F[(3 + i) * 6 + j] = S.B[j * 3 + i];
            F[(3 + i) * 6 + 3 + j] = S.C[si(i, j)];
        }
    R L[21], inv[6];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            R s = F[i * 6 + j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i * (i + 1) / 2 + k] * L[j * (j + 1) / 2 + k];
            if (i == j) {
                R d = sqrt_(s);
                L[i * (i + 1) / 2 + i] = d;
                inv[i] = R(1) / d;
            } else {
                L[i * (i + 1) / 2 + j] = s * inv[j];
            }
        }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        R s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i * (i + 1) / 2 + k] * b[k];
        b[i] = s * inv[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
        R s = b[i];
#pragma unroll
        for (int k = i + 1; k < 6; ++k) s -= L[k * (k + 1) / 2 + i] * b[k];
        b[i] = s * inv[i];
    }
}

// ---------------------------------------------------------------------------
// one dynamics step
// ---------------------------------------------------------------------------
template <typename R> struct StepOut {
    R qdd[NJ];
    R pee[3];      // EE point, world
    R Rn[9];       // last link orientation, world
    R F[6];        // EE wrench estimate [force; moment] (FORCE only)
};

// ext: EXTW_NONE, EXTW_CONST (world wrench F_ext at the EE point, current
// configuration) or EXTW_WALL (the cost's wall model).  tau: joint torques
// (sampled torque plus any joint-space external torque).  v: sampled torque
// for the force estimate (FORCE only).
template <typename R, bool FORCE>
MPPI_HD void dyn_step(const ModelM<R>& M, const CostM<R>& Cst, int ext, const R* q, const R* qd,
                      const R* tau, const R* v, StepOut<R>& out)
{
    R cq[NJ], sq_[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) sincos_(q[i], &sq_[i], &cq[i]);

    // ---- pass 1 (root -> tip): world FK, link velocities, bias forces
    R Rw[9] = {R(1), R(0), R(0), R(0), R(1), R(0), R(0), R(0), R(1)};
    R pw[3] = {R(0), R(0), R(0)};
    R w[3] = {R(0), R(0), R(0)}, vl[3] = {R(0), R(0), R(0)};
    R cc[NJ][4];     // nonzero entries of c_i = v_i x S qd_i: (0,1,3,4)
    R pA[NJ][6];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const LinkM<R>& L = M.L[i];
        R Q[9];
        joint_rot(L.Rp, cq[i], sq_[i], Q);
        R d[3];
        mv3(Rw, L.rp, d);
        pw[0] += d[0]; pw[1] += d[1]; pw[2] += d[2];
        mm3(Rw, Q, Rw);
        // v_i = X_i v_{i-1} + S qd_i
        R rxw[3], t[3];
        cross3(L.rp, w, rxw);
        t[0] = vl[0] - rxw[0]; t[1] = vl[1] - rxw[1]; t[2] = vl[2] - rxw[2];
        mtv3(Q, w, w);
        w[2] += qd[i];
        mtv3(Q, t, vl);
        cc[i][0] = qd[i] * w[1];
        cc[i][1] = -qd[i] * w[0];
        cc[i][2] = qd[i] * vl[1];
        cc[i][3] = -qd[i] * vl[0];
        // h = I v ; pA = v x* h
        R hn[3], hf[3], t1[3], t2[3];
        hn[0] = L.Io[0] * w[0] + L.Io[3] * w[1] + L.Io[4] * w[2];
        hn[1] = L.Io[3] * w[0] + L.Io[1] * w[1] + L.Io[5] * w[2];
        hn[2] = L.Io[4] * w[0] + L.Io[5] * w[1] + L.Io[2] * w[2];
        cross3(L.mc, vl, t1);
        hn[0] += t1[0]; hn[1] += t1[1]; hn[2] += t1[2];
        cross3(L.mc, w, t2);
        hf[0] = L.m * vl[0] - t2[0]; hf[1] = L.m * vl[1] - t2[1]; hf[2] = L.m * vl[2] - t2[2];
        R a[3], b[3], c3[3];
        cross3(w, hn, a);
        cross3(vl, hf, b);
        cross3(w, hf, c3);
        pA[i][0] = a[0] + b[0]; pA[i][1] = a[1] + b[1]; pA[i][2] = a[2] + b[2];
        pA[i][3] = c3[0]; pA[i][4] = c3[1]; pA[i][5] = c3[2];
    }
    {
        R d[3];
        mv3(Rw, M.ree, d);
        out.pee[0] = pw[0] + d[0]; out.pee[1] = pw[1] + d[1]; out.pee[2] = pw[2] + d[2];
#pragma unroll
        for (int i = 0; i < 9; ++i) out.Rn[i] = Rw[i];
    }
    // external wrench on the last link (world force F at the EE point,
    // world moment N): local force f = Rw^T F, moment n = Rw^T N + ree x f
    if (ext != EXTW_NONE) {
        R Fw[3] = {R(0), R(0), R(0)}, Nw[3] = {R(0), R(0), R(0)};
        if (ext == EXTW_WALL) {
            R wxr[3], vel[3], vee[3];
            cross3(w, M.ree, wxr);
            vel[0] = vl[0] + wxr[0]; vel[1] = vl[1] + wxr[1]; vel[2] = vl[2] + wxr[2];
            mv3(Rw, vel, vee);
            R delta = Cst.wall_d0 - dot3(Cst.wall_n, out.pee);
            R ddelta = -dot3(Cst.wall_n, vee);
            R mag = hinge(Cst.wall_k * delta + Cst.wall_c * ddelta);
            Fw[0] = Cst.wall_n[0] * mag; Fw[1] = Cst.wall_n[1] * mag; Fw[2] = Cst.wall_n[2] * mag;
        } else {
            Fw[0] = Cst.F_ext[0]; Fw[1] = Cst.F_ext[1]; Fw[2] = Cst.F_ext[2];
            Nw[0] = Cst.F_ext[3]; Nw[1] = Cst.F_ext[4]; Nw[2] = Cst.F_ext[5];
        }
        R fl[3], nl[3], rf[3];
        mtv3(Rw, Fw, fl);
        mtv3(Rw, Nw, nl);
        cross3(M.ree, fl, rf);
        pA[NJ - 1][0] -= nl[0] + rf[0]; pA[NJ - 1][1] -= nl[1] + rf[1]; pA[NJ - 1][2] -= nl[2] + rf[2];
        pA[NJ - 1][3] -= fl[0]; pA[NJ - 1][4] -= fl[1]; pA[NJ - 1][5] -= fl[2];
    }

    // ---- pass 2 (tip -> root): articulated inertias and bias forces
    R U[NJ][6], iD[NJ], u[NJ], uF[NJ];
    Sym6<R> acc;
#pragma unroll
    for (int i = 0; i < 6; ++i) { acc.A[i] = R(0); acc.C[i] = R(0); }
#pragma unroll
    for (int i = 0; i < 9; ++i) acc.B[i] = R(0);
    R pacc[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    R pF[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int i = NJ - 1; i >= 0; --i) {
        const LinkM<R>& L = M.L[i];
        Sym6<R> IA;
#pragma unroll
        for (int a = 0; a < 6; ++a) IA.A[a] = L.Io[a] + acc.A[a];
        // B = m (c x)
        IA.B[0] = acc.B[0];            IA.B[1] = acc.B[1] - L.mc[2];  IA.B[2] = acc.B[2] + L.mc[1];
        IA.B[3] = acc.B[3] + L.mc[2];  IA.B[4] = acc.B[4];            IA.B[5] = acc.B[5] - L.mc[0];
        IA.B[6] = acc.B[6] - L.mc[1];  IA.B[7] = acc.B[7] + L.mc[0];  IA.B[8] = acc.B[8];
        IA.C[0] = acc.C[0] + L.m; IA.C[1] = acc.C[1] + L.m; IA.C[2] = acc.C[2] + L.m;
        IA.C[3] = acc.C[3];       IA.C[4] = acc.C[4];       IA.C[5] = acc.C[5];
        R p[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) p[a] = pA[i][a] + pacc[a];
        // U = IA S (column 2)
        U[i][0] = IA.A[si(0, 2)]; U[i][1] = IA.A[si(1, 2)]; U[i][2] = IA.A[2];
        U[i][3] = IA.B[6];        U[i][4] = IA.B[7];        U[i][5] = IA.B[8];
        R D = U[i][2] + L.arm;
        iD[i] = R(1) / D;
        u[i] = tau[i] - p[2];
        if (FORCE) uF[i] = v[i] - pF[2];
        if (i > 0) {
            const R* Ui = U[i];
            Sym6<R> Ia;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = a; b < 3; ++b) {
                    Ia.A[si(a, b)] = IA.A[si(a, b)] - Ui[a] * Ui[b] * iD[i];
                    Ia.C[si(a, b)] = IA.C[si(a, b)] - Ui[3 + a] * Ui[3 + b] * iD[i];
                }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int b = 0; b < 3; ++b) Ia.B[a * 3 + b] = IA.B[a * 3 + b] - Ui[a] * Ui[3 + b] * iD[i];
            // pa = p + Ia c + U u / D   (c = (c0, c1, 0, c3, c4, 0))
            R c0 = cc[i][0], c1 = cc[i][1], c3 = cc[i][2], c4 = cc[i][3];
            R uD = u[i] * iD[i];
            R pa[6];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                pa[a] = p[a] + Ia.A[si(a, 0)] * c0 + Ia.A[si(a, 1)] * c1 + Ia.B[a * 3] * c3 +
                        Ia.B[a * 3 + 1] * c4 + Ui[a] * uD;
                pa[3 + a] = p[3 + a] + Ia.B[a] * c0 + Ia.B[3 + a] * c1 + Ia.C[si(a, 0)] * c3 +
                            Ia.C[si(a, 1)] * c4 + Ui[3 + a] * uD;
            }
            R Q[9];
            joint_rot(L.Rp, cq[i], sq_[i], Q);
            congr_force(Q, L.rp, Ia, acc);
            // pacc = X^T pa : f_p = Q f, n_p = Q n + r x f_p
            R fp[3], np_[3], rf[3];
            mv3(Q, pa + 3, fp);
            mv3(Q, pa, np_);
            cross3(L.rp, fp, rf);
            pacc[0] = np_[0] + rf[0]; pacc[1] = np_[1] + rf[1]; pacc[2] = np_[2] + rf[2];
            pacc[3] = fp[0]; pacc[4] = fp[1]; pacc[5] = fp[2];
            if (FORCE) {
                R uFD = uF[i] * iD[i], pf[6];
#pragma unroll
                for (int a = 0; a < 6; ++a) pf[a] = pF[a] + Ui[a] * uFD;
                mv3(Q, pf + 3, fp);
                mv3(Q, pf, np_);
                cross3(L.rp, fp, rf);
                pF[0] = np_[0] + rf[0]; pF[1] = np_[1] + rf[1]; pF[2] = np_[2] + rf[2];
                pF[3] = fp[0]; pF[4] = fp[1]; pF[5] = fp[2];
            }
        }
    }

    // ---- pass 3 (root -> tip): accelerations; force path
    R a[6] = {R(0), R(0), R(0), -M.g[0], -M.g[1], -M.g[2]};
    R aF[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    if (FORCE && Cst.force_mode == 0) { aF[3] = -M.g[0]; aF[4] = -M.g[1]; aF[5] = -M.g[2]; }
    Sym6<R> Om;
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const LinkM<R>& L = M.L[i];
        R Q[9];
        joint_rot(L.Rp, cq[i], sq_[i], Q);
        // a' = X a + c
        R rxw[3], t[3], an[6];
        cross3(L.rp, a, rxw);
        t[0] = a[3] - rxw[0]; t[1] = a[4] - rxw[1]; t[2] = a[5] - rxw[2];
        mtv3(Q, a, an);
        mtv3(Q, t, an + 3);
        an[0] += cc[i][0]; an[1] += cc[i][1]; an[3] += cc[i][2]; an[4] += cc[i][3];
        R Ua = U[i][0] * an[0] + U[i][1] * an[1] + U[i][2] * an[2] + U[i][3] * an[3] +
               U[i][4] * an[4] + U[i][5] * an[5];
        R qddi = (u[i] - Ua) * iD[i];
        out.qdd[i] = qddi;
        an[2] += qddi;
#pragma unroll
        for (int k = 0; k < 6; ++k) a[k] = an[k];
        if (FORCE) {
            cross3(L.rp, aF, rxw);
            t[0] = aF[3] - rxw[0]; t[1] = aF[4] - rxw[1]; t[2] = aF[5] - rxw[2];
            mtv3(Q, aF, an);
            mtv3(Q, t, an + 3);
            R UaF = U[i][0] * an[0] + U[i][1] * an[1] + U[i][2] * an[2] + U[i][3] * an[3] +
                    U[i][4] * an[4] + U[i][5] * an[5];
            an[2] += (uF[i] - UaF) * iD[i];
#pragma unroll
            for (int k = 0; k < 6; ++k) aF[k] = an[k];
            if (i == 0) {
#pragma unroll
                for (int k = 0; k < 6; ++k) { Om.A[k] = R(0); Om.C[k] = R(0); }
#pragma unroll
                for (int k = 0; k < 9; ++k) Om.B[k] = R(0);
                Om.A[2] = iD[0];
            } else {
                Sym6<R> Y;
                congr_motion(Q, L.rp, Om, Y);
                // w = Y U ; beta = U . w
                const R* Ui = U[i];
                R wv[6];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    wv[r] = Y.A[si(r, 0)] * Ui[0] + Y.A[si(r, 1)] * Ui[1] + Y.A[si(r, 2)] * Ui[2] +
                            Y.B[r * 3] * Ui[3] + Y.B[r * 3 + 1] * Ui[4] + Y.B[r * 3 + 2] * Ui[5];
                    wv[3 + r] = Y.B[r] * Ui[0] + Y.B[3 + r] * Ui[1] + Y.B[6 + r] * Ui[2] +
                                Y.C[si(r, 0)] * Ui[3] + Y.C[si(r, 1)] * Ui[4] + Y.C[si(r, 2)] * Ui[5];
                }
                R beta = Ui[0] * wv[0] + Ui[1] * wv[1] + Ui[2] * wv[2] + Ui[3] * wv[3] +
                         Ui[4] * wv[4] + Ui[5] * wv[5];
                R dI = iD[i];
                // Om = Y - (e2 w^T + w e2^T)/D + e2 e2^T (beta/D^2 + 1/D)
                Om = Y;
                Om.A[si(0, 2)] -= wv[0] * dI;
                Om.A[si(1, 2)] -= wv[1] * dI;
                Om.A[2] += (beta * dI - R(2) * wv[2]) * dI + dI;
                Om.B[6] -= wv[3] * dI;
                Om.B[7] -= wv[4] * dI;
                Om.B[8] -= wv[5] * dI;
            }
        }
    }

    if (FORCE) {
        // b = J_n M^-1 tau_F at the last-link origin: remove the propagated
        // base acceleration (pure linear, -R^T g) when gravity was included
        R b[6] = {aF[0], aF[1], aF[2], aF[3], aF[4], aF[5]};
        if (Cst.force_mode == 0) {
            R gl[3];
            mtv3(out.Rn, M.g, gl);
            b[3] += gl[0]; b[4] += gl[1]; b[5] += gl[2];
        }
        chol6_solve(Om, b);   // x = Omega^-1 b  (a spatial force at the link origin)
        // F_ee = T^-T x : F = R f, N = R (n - ree x f)
        R rf[3], nn[3];
        cross3(M.ree, b + 3, rf);
        nn[0] = b[0] - rf[0]; nn[1] = b[1] - rf[1]; nn[2] = b[2] - rf[2];
        mv3(out.Rn, b + 3, out.F);
        mv3(out.Rn, nn, out.F + 3);
    }
}

// EE pose only (terminal cost, tau_ext at x_0)
template <typename R>
MPPI_HD void fk_ee(const ModelM<R>& M, const R* q, R* pee, R* Rn, R* Pj /* [NJ][3] or null */,
                   R* Zj /* [NJ][3] or null */)
{
    R Rw[9] = {R(1), R(0), R(0), R(0), R(1), R(0), R(0), R(0), R(1)};
    R pw[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        R c, s, Q[9], d[3];
        sincos_(q[i], &s, &c);
        joint_rot(M.L[i].Rp, c, s, Q);
        mv3(Rw, M.L[i].rp, d);
        pw[0] += d[0]; pw[1] += d[1]; pw[2] += d[2];
        mm3(Rw, Q, Rw);
        if (Pj) { Pj[i * 3] = pw[0]; Pj[i * 3 + 1] = pw[1]; Pj[i * 3 + 2] = pw[2]; }
        if (Zj) { Zj[i * 3] = Rw[2]; Zj[i * 3 + 1] = Rw[5]; Zj[i * 3 + 2] = Rw[8]; }
    }
    R d[3];
    mv3(Rw, M.ree, d);
    pee[0] = pw[0] + d[0]; pee[1] = pw[1] + d[1]; pee[2] = pw[2] + d[2];
#pragma unroll
    for (int i = 0; i < 9; ++i) Rn[i] = Rw[i];
}

// ---------------------------------------------------------------------------
// cost terms (Eqs. 9-14)
// ---------------------------------------------------------------------------
template <typename R> struct TargetM {
    R p_des[3];
    R RdT[9];     // R_des^T
    R F_des[6];
};

template <typename R>
MPPI_HD R motion_cost(const ModelM<R>& M, const CostM<R>& C, const TargetM<R>& tg, const R* pee, const R* Rn)
{
    R s = C.W_pos[0] * sq(tg.p_des[0] - pee[0]) + C.W_pos[1] * sq(tg.p_des[1] - pee[1]) +
          C.W_pos[2] * sq(tg.p_des[2] - pee[2]);
    if (C.has_ori) {
        R Re[9], Rerr[9], rho[3];
        mm3(Rn, M.Ree, Re);
        mm3(tg.RdT, Re, Rerr);
        so3_log(Rerr, rho);
        s += C.W_ori[0] * rho[0] * rho[0] + C.W_ori[1] * rho[1] * rho[1] + C.W_ori[2] * rho[2] * rho[2];
    }
    return s;
}

template <typename R>
MPPI_HD R joint_cost(const ModelM<R>& M, const CostM<R>& C, const R* q, const R* qd)
{
    R s = R(0);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const LinkM<R>& L = M.L[j];
        s += C.w_q * (sq(hinge(q[j] - L.qmax)) + sq(hinge(L.qmin - q[j])));
        s += C.w_qd * sq(hinge(abs_(qd[j]) - L.qdmax));
        s += C.w_post * sq(q[j] - C.q_rest[j]);
    }
    return s;
}

template <typename R>
MPPI_HD R torque_cost(const ModelM<R>& M, const CostM<R>& C, const R* v)
{
    R s = R(0);
#pragma unroll
    for (int j = 0; j < NJ; ++j) s += C.w_tau * sq(hinge(abs_(v[j]) - M.L[j].taumax));
    return s;
}

template <typename R>
MPPI_HD R force_cost(const CostM<R>& C, const TargetM<R>& tg, const R* F)
{
    R s = R(0);
#pragma unroll
    for (int a = 0; a < 6; ++a) s += C.W_force[a] * sq(tg.F_des[a] - F[a]) + C.W_reg[a] * F[a] * F[a];
    return s;
}

// target from (p_des, quat w x y z, F_des)
template <typename R> MPPI_HD void make_target(const double* tgt, TargetM<R>& tg)
{
    double w = tgt[3], x = tgt[4], y = tgt[5], z = tgt[6];
    double n = std::sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    double Rd[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                    2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                    2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) tg.RdT[i * 3 + j] = R(Rd[j * 3 + i]);
    for (int a = 0; a < 3; ++a) tg.p_des[a] = R(tgt[a]);
    for (int a = 0; a < 6; ++a) tg.F_des[a] = R(tgt[7 + a]);
}

// tau_ext = J(q0)^T F_ext for the constant external wrench (Sec. III-A:
// held over the whole horizon).  (J^T F)_j = (z_j x (p_ee - p_j)).F + z_j.N
template <typename R> MPPI_HD void const_ext_torque(const ModelM<R>& M, const CostM<R>& C, const R* q0, R* tau_ext)
{
    R pee[3], Rn[9], P[NJ * 3], Z[NJ * 3];
    fk_ee(M, q0, pee, Rn, P, Z);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        R d[3] = {pee[0] - P[j * 3], pee[1] - P[j * 3 + 1], pee[2] - P[j * 3 + 2]}, c[3];
        cross3(Z + j * 3, d, c);
        tau_ext[j] = dot3(c, C.F_ext) + dot3(Z + j * 3, C.F_ext + 3);
    }
}

}  // namespace mppi
