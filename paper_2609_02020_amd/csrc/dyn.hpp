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
//     F_ee = Lambda J M^-1 tau_F, from the articulated-body factors
//     (U_i, D_i) of the same step: J_n M^-1 J_n^T = A A^T with one column
//     of A per joint, carried outward link by link, and J_n M^-1 tau_F =
//     A y from one extra zero-velocity pass with the same factors; the
//     wrench is the least-squares solution of A^T x = y (lsq_wrench,
//     modified Gram-Schmidt), which keeps FP32 accurate near kinematic
//     singularities where forming Lambda^-1 would not, and
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
// FP32 on the device: the hardware sine/cosine, whose input is in
// revolutions (argument / 2 pi); joint angles stay far inside its range.
MPPI_HD void sincos_(float x, float* s, float* c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    const float rev = x * 0.15915494309189535f;
    *s = __builtin_amdgcn_sinf(rev);
    *c = __builtin_amdgcn_cosf(rev);
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
    const float rev = 0.5f * x;
    *s = __builtin_amdgcn_sinf(rev);
    *c = __builtin_amdgcn_cosf(rev);
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
MPPI_HD float log_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_logf(x) * 0.69314718055994531f;   // hardware log2
#else
    return std::log(x);
#endif
}
MPPI_HD double log_(double x) { return std::log(x); }
MPPI_HD float atan2_(float y, float x) { return std::atan2(y, x); }
MPPI_HD double atan2_(double y, double x) { return std::atan2(y, x); }
MPPI_HD float abs_(float x) { return std::fabs(x); }
MPPI_HD double abs_(double x) { return std::fabs(x); }

MPPI_HD float fma_(float a, float b, float c) { return std::fma(a, b, c); }
MPPI_HD double fma_(double a, double b, double c) { return std::fma(a, b, c); }
// reciprocal / square root: the single-rounding hardware instructions in
// FP32 (1 ulp), exact IEEE operations in FP64
MPPI_HD float rcp_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}
MPPI_HD double rcp_(double x) { return 1.0 / x; }
MPPI_HD float rsqrt_sqrt_(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return std::sqrt(x);
#endif
}
MPPI_HD double rsqrt_sqrt_(double x) { return std::sqrt(x); }
// keeps the instruction scheduler from moving code across this point (on
// the device; nothing on the host): placed after a batch of LDS or memory
// reads, it keeps the batch issued together ahead of its uses
MPPI_HD void sched_fence()
{
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_sched_barrier(0);
#endif
}
MPPI_HD float max0_(float x) { return std::fmax(x, 0.0f); }
MPPI_HD double max0_(double x) { return std::fmax(x, 0.0); }

template <typename R> MPPI_HD R hinge(R x) { return max0_(x); }
template <typename R> MPPI_HD R sq(R x) { return x * x; }

// ---------------------------------------------------------------------------
// model and cost as the kernels read them
// ---------------------------------------------------------------------------
template <typename R> struct LinkM {
    R Rp[9];      // R_parent, row-major
    R rp[3];      // r_parent
    R Ic[6];      // inertia about the CoM, link-frame axes (xx yy zz xy xz yz)
    R com[3];     // CoM in the link frame
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
    // time correlation of the perturbation: du_t = rho du_{t-1} + sig_c z_t
    // for t >= 1 with sig_c = sqrt(1 - rho^2) sigma (rho = 0: i.i.d.)
    R rho;
    R sig_c[NJ];
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
    // collision term (Eqs. 14-15)
    R w_coll;
    R obs[4][6];      // obstacle segments, world
    R dth2[32];       // squared thresholds
    int n_pairs;
    int pa[32], pb[32];   // segment ids: 0..NJ-1 links, NJ + o obstacle o
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
template <typename R> struct Sym6 {
    R A[6];
    R B[9];
    R C[6];
};

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
    R rad = rsqrt_sqrt_(R(-2) * log_(ua));
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

// Least-squares form of the wrench solve of Eq. 13.  With the inverse
// operational-space inertia factored as Omega = A A^T (A: 6 x 7, one column
// per joint) and J M^-1 tau_F = A y, the wrench x = Omega^-1 A y is the
// minimiser of |A^T x - y|.  Modified Gram-Schmidt on the columns of
// [A^T | y] (the right-hand side taken through the same projections, the
// augmented form that Bjorck showed backward stable for least squares)
// gives A^T = Q Rm and Q^T y, then x = Rm^-1 Q^T y.  Its rounding error
// grows with cond(A) = cond(Omega)^(1/2), where forming Omega and solving
// it (the normal equations) grows with cond(Omega), which near a kinematic
// singularity exceeds 1 / u in FP32.  At: rows = joints, columns = the six
// wrench components; At and y are overwritten.
template <typename R> MPPI_HD void lsq_wrench(R (&At)[NJ][6], R (&y)[NJ], R* x)
{
    R Rm[6][6], z[6], id[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        R n2 = R(0);
#pragma unroll
        for (int i = 0; i < NJ; ++i) n2 = fma_(At[i][s], At[i][s], n2);
        const R r = rsqrt_sqrt_(n2);
        id[s] = rcp_(r);
        R qv[NJ];
#pragma unroll
        for (int i = 0; i < NJ; ++i) qv[i] = At[i][s] * id[s];
#pragma unroll
        for (int c = s + 1; c < 6; ++c) {
            R d = R(0);
#pragma unroll
            for (int i = 0; i < NJ; ++i) d = fma_(qv[i], At[i][c], d);
            Rm[s][c] = d;
#pragma unroll
            for (int i = 0; i < NJ; ++i) At[i][c] = fma_(-d, qv[i], At[i][c]);
        }
        R d = R(0);
#pragma unroll
        for (int i = 0; i < NJ; ++i) d = fma_(qv[i], y[i], d);
        z[s] = d;
#pragma unroll
        for (int i = 0; i < NJ; ++i) y[i] = fma_(-d, qv[i], y[i]);
    }
#pragma unroll
    for (int s = 5; s >= 0; --s) {
        R t = z[s];
#pragma unroll
        for (int c = s + 1; c < 6; ++c) t = fma_(-Rm[s][c], x[c], t);
        x[s] = t * id[s];
    }
}

// ---------------------------------------------------------------------------
// one dynamics step: articulated-body algorithm in world-aligned frames
// centred on the joints
// ---------------------------------------------------------------------------
// Frame i has world axes and its origin at joint i's origin p_i; spatial
// vectors are [angular; linear] about p_i.  Joint i then has the motion
// subspace S_i = (z_i, 0), and moving between links is a pure translation
// by r_i = p_i - p_{i-1} (no rotation):
//   motion  (w, v) at p_{i-1} -> (w, v + w x r_i) at p_i
//   force   (n, f) at p_{i+1} -> (n + r_{i+1} x f, f) at p_i
// The spatial inertia of link i about p_i is
//   I_i = [Ibar_c + m (|c|^2 1 - c c^T),  m c x;  (m c x)^T,  m 1],
// Ibar_c = R_i I_c R_i^T, c = R_i com (CoM relative to p_i).  Moment arms
// stay at link length, which keeps FP32 rounding at the level of a
// link-local formulation while avoiding its per-link rotations.
//   pass 1 (root->tip): v_i = X_i v_{i-1} + S_i qd_i, c_i = v_i x S_i qd_i,
//                       p_i = v_i x* I_i v_i - f_ext,i
//   pass 2 (tip->root): IA_i = I_i + X_{i+1}^T Ia_{i+1} X_{i+1},
//                       pA_i = p_i + X_{i+1}^T pa_{i+1},
//                       U_i = IA_i S_i, D_i = S_i.U_i + a_i, u_i = tau_i - S_i.pA_i,
//                       Ia_i = IA_i - U_i U_i^T / D_i, pa_i = pA_i + Ia_i c_i + U_i u_i / D_i
//   pass 3 (root->tip): a'_i = X_i a_{i-1} + c_i, qdd_i = (u_i - U_i.a'_i) / D_i,
//                       a_i = a'_i + S_i qdd_i, a_{-1} = (0, -g)
// Force path (Eq. 13): Omega_i = P_i X_i Omega_{i-1} X_i^T P_i^T + S_i S_i^T / D_i,
// P_i = 1 - S_i U_i^T / D_i, Omega_{-1} = 0, gives Omega_n = J_n M^-1 J_n^T
// about p_n, a sum of one rank-one term per joint (force_estimate carries
// its factor A instead of Omega); a zero-velocity solve with torques tau_F
// gives b = J_n M^-1 tau_F; x = Omega_n^-1 b is the spatial force about p_n
// and the EE wrench is F = x_f, N = x_n - (p_ee - p_n) x x_f.
// What the force estimate needs from one articulated-body step: the joint
// axes, the link translations r_0..r_6, the factors U_i and 1/D_i and the
// EE offset from p_n (all world axes).  force_estimate() turns it, with the
// sampled torques, into F_ee.
template <typename R> struct ForceIn {
    R z[NJ][3];
    R rr[NJ][3];
    R U[NJ][6];
    R iD[NJ];
    R ree[3];
};
// Flat layout of a ForceIn for a handoff through memory (index of each
// value): 94 values.
constexpr int kFiZ = 0, kFiRr = 21, kFiU = 42, kFiD = 84, kFiRee = 91, kFiCount = 94;

template <typename R> struct StepOut {
    R qdd[NJ];
    R pee[3];      // EE point, world
    R Rn[9];       // last link orientation, world
    R F[6];        // EE wrench estimate [force; moment] (FORCE only)
};

template <typename R> MPPI_HD void sym6_mv(const Sym6<R>& M, const R* x, R* y)
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        y[a] = M.A[si(a, 0)] * x[0] + M.A[si(a, 1)] * x[1] + M.A[si(a, 2)] * x[2] +
               M.B[a * 3] * x[3] + M.B[a * 3 + 1] * x[4] + M.B[a * 3 + 2] * x[5];
        y[3 + a] = M.B[a] * x[0] + M.B[3 + a] * x[1] + M.B[6 + a] * x[2] +
                   M.C[si(a, 0)] * x[3] + M.C[si(a, 1)] * x[4] + M.C[si(a, 2)] * x[5];
    }
}
template <typename R> MPPI_HD R dot6(const R* a, const R* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}
// M += x y^T + y x^T (symmetric storage)
// M -= U W^T for W = U / D (symmetric result): one fma per stored entry
template <typename R> MPPI_HD void sym6_sub_outer(Sym6<R>& M, const R* U, const R* W)
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = a; b < 3; ++b) {
            M.A[si(a, b)] = fma_(-U[a], W[b], M.A[si(a, b)]);
            M.C[si(a, b)] = fma_(-U[3 + a], W[3 + b], M.C[si(a, b)]);
        }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) M.B[a * 3 + b] = fma_(-U[a], W[3 + b], M.B[a * 3 + b]);
}
// Force-side shift of a symmetric spatial matrix from a reference point p'
// to p = p' - r (r = p' - p): out = X^T M X with X = [1 0; -rx 1]:
//   C' = C, B' = B + rx C, A' = A + rx B^T + (rx B^T)^T - rx C rx.
// (rx M)_ij = r_{i+1} M_{i+2,j} - r_{i+2} M_{i+1,j} (indices mod 3).
template <typename R> MPPI_HD void shift_force(const R* r, Sym6<R>& M)
{
    R Cf[9], P[9], G[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Cf[i * 3 + j] = M.C[si(i, j)];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            P[i * 3 + j] = fma_(r[i1], Cf[i2 * 3 + j], -r[i2] * Cf[i1 * 3 + j]);          // rx C
            G[i * 3 + j] = fma_(r[i1], M.B[j * 3 + i2], -r[i2] * M.B[j * 3 + i1]);      // rx B^T
        }
    }
    // A'_ij = A_ij + G_ij + G_ji - (P rx)_ij, (P rx)_ij = P_{i,j+1} r_{j+2} - P_{i,j+2} r_{j+1}
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            R acc = M.A[si(i, j)] + G[i * 3 + j] + G[j * 3 + i];
            acc = fma_(P[i * 3 + j2], r[j1], acc);
            M.A[si(i, j)] = fma_(-P[i * 3 + j1], r[j2], acc);
        }
#pragma unroll
    for (int i = 0; i < 9; ++i) M.B[i] += P[i];
}
// EE wrench estimate of Eq. 13 from the factors of one step and the
// sampled torques v, as the least-squares problem of lsq_wrench:
//   uF_i = tau_F,i - S_i.pF by the tip-to-root pass of a zero-velocity
//       articulated-body solve with the same factors (pF += U_i uF_i / D_i,
//       shifted to the parent);
//   the columns c_i = T_i S_i of the factorisation
//       Omega_n = J_n M^-1 J_n^T = sum_i c_i c_i^T / D_i,
//       T_i = P_n X_n ... P_{i+1} X_{i+1},  P_k = 1 - S_k U_k^T / D_k,
//       carried link by link from the root (every earlier column shifted to
//       p_k and projected by P_k, then c_k = S_k appended);
//   J_n M^-1 tau_F = sum_i c_i (uF_i - U_i.a_b) / D_i, where a_b = (0, -g)
//       when tau_F = v - g(q) (force_mode 0: the gravity torque enters as the
//       rigid base acceleration -g, whose projections telescope into the
//       U_i.a_b terms) and a_b = 0 for tau_F = v;
// so A = [c_i / sqrt(D_i)] and y_i = (uF_i - U_i.a_b) / sqrt(D_i).  The
// solution x is the spatial force about p_n and F = (x_f, x_n - ree x x_f).
template <typename R>
MPPI_HD void force_estimate(const ForceIn<R>& fi, const R* v, const R* g, int force_mode, R* F)
{
    R uF[NJ];
    R pF[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int i = NJ - 1; i >= 0; --i) {
        uF[i] = v[i] - dot3(fi.z[i], pF);
        if (i > 0) {
            const R uFD = uF[i] * fi.iD[i];
#pragma unroll
            for (int a = 0; a < 6; ++a) pF[a] += fi.U[i][a] * uFD;
            R rf[3];
            cross3(fi.rr[i], pF + 3, rf);
            pF[0] += rf[0]; pF[1] += rf[1]; pF[2] += rf[2];
        }
    }
    R At[NJ][6], y[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        // earlier columns: shift from p_{i-1} to p_i, then project by P_i
#pragma unroll
        for (int l = 0; l < i; ++l) {
            R wxr[3];
            cross3(At[l], fi.rr[i], wxr);
            At[l][3] += wxr[0]; At[l][4] += wxr[1]; At[l][5] += wxr[2];
            const R pr = dot6(fi.U[i], At[l]) * fi.iD[i];
            At[l][0] = fma_(-fi.z[i][0], pr, At[l][0]);
            At[l][1] = fma_(-fi.z[i][1], pr, At[l][1]);
            At[l][2] = fma_(-fi.z[i][2], pr, At[l][2]);
        }
        At[i][0] = fi.z[i][0]; At[i][1] = fi.z[i][1]; At[i][2] = fi.z[i][2];
        At[i][3] = R(0); At[i][4] = R(0); At[i][5] = R(0);
        R ub = uF[i];
        if (force_mode == 0) ub += fi.U[i][3] * g[0] + fi.U[i][4] * g[1] + fi.U[i][5] * g[2];
        y[i] = ub;
    }
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const R sD = rsqrt_sqrt_(fi.iD[i]);
#pragma unroll
        for (int a = 0; a < 6; ++a) At[i][a] *= sD;
        y[i] *= sD;
    }
    R x[6];
    lsq_wrench(At, y, x);   // spatial force about p_n
    R rf[3];
    cross3(fi.ree, x + 3, rf);
    F[0] = x[3]; F[1] = x[4]; F[2] = x[5];
    F[3] = x[0] - rf[0]; F[4] = x[1] - rf[1]; F[5] = x[2] - rf[2];
}

// ext: EXTW_NONE, EXTW_CONST (world wrench F_ext at the EE point, current
// configuration) or EXTW_WALL (the cost's wall model).  tau: joint torques
// (sampled torque plus any joint-space external torque).  v: sampled torque
// for the force estimate (FORCE only).
// hand (FORCE only): when non-null, the inputs of the force estimate are
// stored there in the flat ForceIn layout, value f at hand[f * hstride],
// each as soon as the step no longer needs it, and out.F is left unset.
template <typename R, bool FORCE>
MPPI_HD void dyn_step(const ModelM<R>& M, const CostM<R>& Cst, int ext, const R* q, const R* qd,
                      const R* tau, const R* v, StepOut<R>& out, R* hand = nullptr, int hstride = 0)
{
    R z[NJ][3];      // joint axes (world)
    R rr[NJ][3];     // p_i - p_{i-1} (r_0 = p_0)
    R cc[NJ][6];     // velocity-product accelerations, about p_i
    R pA[NJ][6];     // bias forces, about p_i
    R Iw[NJ][6];     // rotational inertia about p_i, world axes (sym storage)
    R mc[NJ][3];     // m c, c = CoM - p_i

    // ---- pass 1 (root -> tip)
    R Rw[9] = {R(1), R(0), R(0), R(0), R(1), R(0), R(0), R(0), R(1)};
    R pw[3] = {R(0), R(0), R(0)};
    R vw[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const LinkM<R>& L = M.L[i];
        R c, s, Q[9];
        sincos_(q[i], &s, &c);
        joint_rot(L.Rp, c, s, Q);
        mv3(Rw, L.rp, rr[i]);
        pw[0] += rr[i][0]; pw[1] += rr[i][1]; pw[2] += rr[i][2];
        mm3(Rw, Q, Rw);
        z[i][0] = Rw[2]; z[i][1] = Rw[5]; z[i][2] = Rw[8];
        // link inertia about p_i in world axes
        R cw[3], Ic[6];
        mv3(Rw, L.com, cw);
        congr_sym3<false>(Rw, L.Ic, Ic);
        const R c2 = dot3(cw, cw);
        Iw[i][0] = Ic[0] + L.m * (c2 - cw[0] * cw[0]);
        Iw[i][1] = Ic[1] + L.m * (c2 - cw[1] * cw[1]);
        Iw[i][2] = Ic[2] + L.m * (c2 - cw[2] * cw[2]);
        Iw[i][3] = Ic[3] - L.m * cw[0] * cw[1];
        Iw[i][4] = Ic[4] - L.m * cw[0] * cw[2];
        Iw[i][5] = Ic[5] - L.m * cw[1] * cw[2];
        mc[i][0] = L.m * cw[0]; mc[i][1] = L.m * cw[1]; mc[i][2] = L.m * cw[2];
        // v_i = X_i v_{i-1} + S_i qd_i  (shift by r_i, then the joint rate)
        R wxr[3];
        cross3(vw, rr[i], wxr);
        vw[3] += wxr[0]; vw[4] += wxr[1]; vw[5] += wxr[2];
        const R sw[3] = {z[i][0] * qd[i], z[i][1] * qd[i], z[i][2] * qd[i]};
        vw[0] += sw[0]; vw[1] += sw[1]; vw[2] += sw[2];
        // c_i = v_i x (S_i qd_i) = (w x sw, v x sw)
        R t1[3], t2[3], t3[3];
        cross3(vw, sw, t1);
        cross3(vw + 3, sw, t2);
        cc[i][0] = t1[0]; cc[i][1] = t1[1]; cc[i][2] = t1[2];
        cc[i][3] = t2[0]; cc[i][4] = t2[1]; cc[i][5] = t2[2];
        // h = I v ; p = v x* h = (w x hn + v x hf, w x hf)
        R hn[3], hf[3], u1[3], u2[3];
        hn[0] = Iw[i][0] * vw[0] + Iw[i][3] * vw[1] + Iw[i][4] * vw[2];
        hn[1] = Iw[i][3] * vw[0] + Iw[i][1] * vw[1] + Iw[i][5] * vw[2];
        hn[2] = Iw[i][4] * vw[0] + Iw[i][5] * vw[1] + Iw[i][2] * vw[2];
        cross3(mc[i], vw + 3, u1);
        hn[0] += u1[0]; hn[1] += u1[1]; hn[2] += u1[2];
        cross3(mc[i], vw, u2);
        hf[0] = L.m * vw[3] - u2[0]; hf[1] = L.m * vw[4] - u2[1]; hf[2] = L.m * vw[5] - u2[2];
        cross3(vw, hn, t1);
        cross3(vw + 3, hf, t2);
        cross3(vw, hf, t3);
        pA[i][0] = t1[0] + t2[0]; pA[i][1] = t1[1] + t2[1]; pA[i][2] = t1[2] + t2[2];
        pA[i][3] = t3[0]; pA[i][4] = t3[1]; pA[i][5] = t3[2];
    }
    R ree_w[3];   // EE point relative to p_n
    mv3(Rw, M.ree, ree_w);
    out.pee[0] = pw[0] + ree_w[0]; out.pee[1] = pw[1] + ree_w[1]; out.pee[2] = pw[2] + ree_w[2];
#pragma unroll
    for (int i = 0; i < 9; ++i) out.Rn[i] = Rw[i];
    // external wrench on the last link: world force F at the EE point and
    // world moment N, about p_n: (N + ree_w x F, F)
    if (ext != EXTW_NONE) {
        R Fw[3] = {R(0), R(0), R(0)}, Nw[3] = {R(0), R(0), R(0)};
        if (ext == EXTW_WALL) {
            R wxr[3];
            cross3(vw, ree_w, wxr);
            const R vee[3] = {vw[3] + wxr[0], vw[4] + wxr[1], vw[5] + wxr[2]};
            R delta = Cst.wall_d0 - dot3(Cst.wall_n, out.pee);
            R ddelta = -dot3(Cst.wall_n, vee);
            R mag = hinge(Cst.wall_k * delta + Cst.wall_c * ddelta);
            Fw[0] = Cst.wall_n[0] * mag; Fw[1] = Cst.wall_n[1] * mag; Fw[2] = Cst.wall_n[2] * mag;
        } else {
            Fw[0] = Cst.F_ext[0]; Fw[1] = Cst.F_ext[1]; Fw[2] = Cst.F_ext[2];
            Nw[0] = Cst.F_ext[3]; Nw[1] = Cst.F_ext[4]; Nw[2] = Cst.F_ext[5];
        }
        R rf[3];
        cross3(ree_w, Fw, rf);
        pA[NJ - 1][0] -= Nw[0] + rf[0]; pA[NJ - 1][1] -= Nw[1] + rf[1]; pA[NJ - 1][2] -= Nw[2] + rf[2];
        pA[NJ - 1][3] -= Fw[0]; pA[NJ - 1][4] -= Fw[1]; pA[NJ - 1][5] -= Fw[2];
    }

    // ---- pass 2 (tip -> root)
    R U[NJ][6], iD[NJ], u[NJ];
    Sym6<R> IA;
#pragma unroll
    for (int a = 0; a < 6; ++a) { IA.A[a] = R(0); IA.C[a] = R(0); }
#pragma unroll
    for (int a = 0; a < 9; ++a) IA.B[a] = R(0);
    R pacc[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int i = NJ - 1; i >= 0; --i) {
        const LinkM<R>& L = M.L[i];
        // IA_i = I_i + (child contribution, already about p_i)
#pragma unroll
        for (int a = 0; a < 6; ++a) IA.A[a] += Iw[i][a];
        IA.B[1] -= mc[i][2]; IA.B[2] += mc[i][1];
        IA.B[3] += mc[i][2]; IA.B[5] -= mc[i][0];
        IA.B[6] -= mc[i][1]; IA.B[7] += mc[i][0];
        IA.C[0] += L.m; IA.C[1] += L.m; IA.C[2] += L.m;
        R p[6];
#pragma unroll
        for (int a = 0; a < 6; ++a) p[a] = pA[i][a] + pacc[a];
        // U = IA S = (A z, B^T z), D = z.(A z) + a
        const R* zi = z[i];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            U[i][a] = IA.A[si(a, 0)] * zi[0] + IA.A[si(a, 1)] * zi[1] + IA.A[si(a, 2)] * zi[2];
            U[i][3 + a] = IA.B[a] * zi[0] + IA.B[3 + a] * zi[1] + IA.B[6 + a] * zi[2];
        }
        iD[i] = rcp_(dot3(zi, U[i]) + L.arm);
        u[i] = tau[i] - dot3(zi, p);
        if (i > 0) {
            R UD[6];
#pragma unroll
            for (int a = 0; a < 6; ++a) UD[a] = U[i][a] * iD[i];
            sym6_sub_outer(IA, U[i], UD);        // Ia = IA - U U^T / D
            R Iac[6];
            sym6_mv(IA, cc[i], Iac);
            const R uD = u[i] * iD[i];
#pragma unroll
            for (int a = 0; a < 6; ++a) pacc[a] = p[a] + Iac[a] + U[i][a] * uD;
            // move Ia and pa to p_{i-1}: force shift by r_i
            shift_force(rr[i], IA);
            R rf[3];
            cross3(rr[i], pacc + 3, rf);
            pacc[0] += rf[0]; pacc[1] += rf[1]; pacc[2] += rf[2];
        }
    }

    // ---- pass 3 (root -> tip)
    R a[6] = {R(0), R(0), R(0), -M.g[0], -M.g[1], -M.g[2]};
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        // a' = X a + c
        R wxr[3];
        cross3(a, rr[i], wxr);
        R an[6] = {a[0] + cc[i][0], a[1] + cc[i][1], a[2] + cc[i][2],
                   a[3] + wxr[0] + cc[i][3], a[4] + wxr[1] + cc[i][4], a[5] + wxr[2] + cc[i][5]};
        const R qddi = (u[i] - dot6(U[i], an)) * iD[i];
        out.qdd[i] = qddi;
        a[0] = an[0] + z[i][0] * qddi; a[1] = an[1] + z[i][1] * qddi; a[2] = an[2] + z[i][2] * qddi;
        a[3] = an[3]; a[4] = an[4]; a[5] = an[5];
        if (FORCE && hand) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                hand[(kFiZ + 3 * i + c) * hstride] = z[i][c];
                hand[(kFiRr + 3 * i + c) * hstride] = rr[i][c];
            }
#pragma unroll
            for (int c = 0; c < 6; ++c) hand[(kFiU + 6 * i + c) * hstride] = U[i][c];
            hand[(kFiD + i) * hstride] = iD[i];
        }
    }

    if (FORCE && hand) {
#pragma unroll
        for (int c = 0; c < 3; ++c) hand[(kFiRee + c) * hstride] = ree_w[c];
    } else if (FORCE) {
        ForceIn<R> fi;
#pragma unroll
        for (int i = 0; i < NJ; ++i) {
#pragma unroll
            for (int c = 0; c < 3; ++c) { fi.z[i][c] = z[i][c]; fi.rr[i][c] = rr[i][c]; }
#pragma unroll
            for (int c = 0; c < 6; ++c) fi.U[i][c] = U[i][c];
            fi.iD[i] = iD[i];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) fi.ree[c] = ree_w[c];
        force_estimate(fi, v, M.g, Cst.force_mode, out.F);
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
// collision term (Eqs. 14-15)
// ---------------------------------------------------------------------------
MPPI_HD int uniform_(int x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_readfirstlane(x);   // the same in every lane
#else
    return x;
#endif
}
template <typename R> MPPI_HD R clamp01_(R x) { return x < R(0) ? R(0) : (x > R(1) ? R(1) : x); }

// Squared minimum distance between segments [a0, a1] and [b0, b1] (the
// closest-point construction of Lumelsky's method): the line-line optimum
// s clamped to [0, 1] (0 for parallel lines), t optimal for that s, and if
// t leaves [0, 1] it is clamped and s re-optimised for it.  Every candidate
// is formed and the case picked by selects, with one reciprocal per
// denominator (the lanes of a wave take different cases; branches would
// run them one after another).
template <typename R> MPPI_HD R seg_dist2(const R* a0, const R* a1, const R* b0, const R* b1)
{
    R da[3], db[3], r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) { da[c] = a1[c] - a0[c]; db[c] = b1[c] - b0[c]; r[c] = a0[c] - b0[c]; }
    const R A = dot3(da, da), B = dot3(da, db), E = dot3(db, db), Cr = dot3(da, r), F = dot3(db, r);
    const R den = A * E - B * B;
    // 1 / A, 1 / E, 1 / den, or 0 where the denominator vanishes (a point
    // segment, parallel lines): the candidates that divide by it become 0
    const R rA = A > R(0) ? rcp_(A) : R(0);
    const R rE = E > R(0) ? rcp_(E) : R(0);
    const R rD = den > R(0) ? rcp_(den) : R(0);
    const R s_lo = clamp01_(-Cr * rA);        // s re-optimised for t = 0
    const R s_hi = clamp01_((B - Cr) * rA);   // for t = 1
    const R s_in = clamp01_((B * F - Cr * E) * rD);
    const R t_in = (B * s_in + F) * rE;
    const bool pt = !(E > R(0));              // b is a point: t = 0
    const bool lo = pt || t_in < R(0), hi = !pt && t_in > R(1);
    const R t = lo ? R(0) : (hi ? R(1) : t_in);
    const R s = lo ? s_lo : (hi ? s_hi : s_in);
    R e[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) e[c] = r[c] + s * da[c] - t * db[c];
    return dot3(e, e);
}

// ends of segment `id` (uniform): link id from joint origin P[id] to
// P[id + 1] (P[NJ] = EE point), else obstacle id - NJ
template <typename R>
MPPI_HD void seg_ends(int id, const R (&P)[NJ + 1][3], const CostM<R>& C, R* e0, R* e1)
{
    switch (id) {
#define MPPI_LINK_SEG(i)                                                                    \
    case i:                                                                                 \
        for (int c = 0; c < 3; ++c) { e0[c] = P[i][c]; e1[c] = P[i + 1][c]; }              \
        return;
        MPPI_LINK_SEG(0) MPPI_LINK_SEG(1) MPPI_LINK_SEG(2) MPPI_LINK_SEG(3)
        MPPI_LINK_SEG(4) MPPI_LINK_SEG(5) MPPI_LINK_SEG(6)
#undef MPPI_LINK_SEG
    default:
        for (int c = 0; c < 3; ++c) { e0[c] = C.obs[id - NJ][c]; e1[c] = C.obs[id - NJ][3 + c]; }
    }
}

// C_collision(q) = w_collision * #{pairs i: d_i < d_th,i}, compared as
// squared distances
template <typename R>
MPPI_HD R collision_cost(const ModelM<R>& M, const CostM<R>& C, const R* q);

// ---------------------------------------------------------------------------
// cost terms (Eqs. 9-14)
// ---------------------------------------------------------------------------
template <typename R>
MPPI_HD R collision_cost(const ModelM<R>& M, const CostM<R>& C, const R* q)
{
    R P[NJ + 1][3], Rn[9];
    fk_ee(M, q, P[NJ], Rn, &P[0][0], (R*)nullptr);
    R hits = R(0);
    const int np = uniform_(C.n_pairs);
    for (int i = 0; i < np; ++i) {
        R a0[3], a1[3], b0[3], b1[3];
        seg_ends(uniform_(C.pa[i]), P, C, a0, a1);
        seg_ends(uniform_(C.pb[i]), P, C, b0, b1);
        if (seg_dist2(a0, a1, b0, b1) < C.dth2[i]) hits += R(1);
    }
    return C.w_coll * hits;
}

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
// Joint torques J(q)^T W of a world wrench W = [force; moment] acting at
// the EE point (Eq. 5's tau_ext for a wrench at the EE).
template <typename R> MPPI_HD void ee_wrench_torque(const ModelM<R>& M, const R* q, const R* W, R* tau)
{
    R pee[3], Rn[9], P[NJ * 3], Z[NJ * 3];
    fk_ee(M, q, pee, Rn, P, Z);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        R d[3] = {pee[0] - P[j * 3], pee[1] - P[j * 3 + 1], pee[2] - P[j * 3 + 2]}, c[3];
        cross3(Z + j * 3, d, c);
        tau[j] = dot3(c, W) + dot3(Z + j * 3, W + 3);
    }
}
template <typename R> MPPI_HD void const_ext_torque(const ModelM<R>& M, const CostM<R>& C, const R* q0, R* tau_ext)
{
    ee_wrench_torque(M, q0, C.F_ext, tau_ext);
}

}  // namespace mppi
