// rollout.hpp -- one MPPI sample rolled out over the horizon (Sec. II Eq. 3
// with the dynamics of Sec. III-A and the cost of Sec. III-B):
//   for t = 0 .. T-1:
//     du_t = sigma * z(seed, tick, k, t)            (Eq. 2, Philox + Box-Muller;
//            for t >= 1 rho du_{t-1} + sqrt(1 - rho^2) sigma z when the
//            perturbation is correlated in time, noise_step below)
//     v_t  = u_t + du_t
//     S   += l(x_t, v_t)                            (Eqs. 9-14, pre-step state)
//     qdd  = M^-1 (v_t + tau_ext - h)               (Eq. 6, articulated-body)
//     qd  += qdd dt ; q += qd dt                    (Eq. 7 as written)
//   S += phi(x_T) = w_T (C_pos + C_ori + C_joint)(x_T)
// The cost is accumulated in the rollout precision R.
#pragma once

#include "dyn.hpp"
#include "dyn_m.hpp"

namespace mppi {

template <typename R> MPPI_HD bool finite_(R x) { return x - x == R(0); }

// The same object behind an address the compiler cannot prove loop-invariant,
// so that reads of model and cost constants stay inside the step loop
// (re-read each step from the scalar cache or LDS) instead of being hoisted
// and held in registers for the whole rollout.
template <typename T> MPPI_HD const T* per_step(const T* p)
{
#if defined(__HIP_DEVICE_COMPILE__)
    int off = 0;
    asm volatile("" : "+s"(off));
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off);
#else
    return p;
#endif
}

// The perturbation of step t from that step's normals z, updating du (the
// previous step's perturbation) in place: sigma z at t = 0, then
// rho du + sqrt(1 - rho^2) sigma z, a stationary AR(1) process in time with
// the variance sigma^2 of Eq. 2 at every step.  rho = 0 leaves the
// independent draws of Eq. 2 (and skips the recursion: one uniform branch).
template <typename R> MPPI_HD void noise_step(const CostM<R>& C, const R* z, R* du, int t)
{
    if (t == 0 || C.rho == R(0)) {
#pragma unroll
        for (int j = 0; j < NJ; ++j) du[j] = C.sigma[j] * z[j];
    } else {
#pragma unroll
        for (int j = 0; j < NJ; ++j) du[j] = C.rho * du[j] + C.sig_c[j] * z[j];
    }
}

// noise_out / noise_lds (either may be null) receive du[t][j] at
// (t*7 + j) * stride.
// EXPLICIT selects the paper's own dynamics route (dyn_m.hpp: M by Eq. 8,
// Cholesky solve) instead of the articulated-body step; COLL adds the
// collision term (a compile-time switch: its code in the step loop slows
// the rollouts that do not use it).
template <typename R, bool FORCE, bool EXPLICIT = false, bool COLL = false, typename UT>
MPPI_HD R rollout_sample(const ModelM<R>& Mc, const CostM<R>& Cc, const TargetM<R>& tg,
                         const R* q0, const R* qd0, const R* tau_ext_c, const UT* U_nom, int T,
                         uint64_t seed, uint32_t tick, uint32_t k, R* noise_out, size_t noise_stride,
                         R* noise_lds = nullptr, int lds_stride = 0)
{
    R q[NJ], qd[NJ], du[NJ], S = R(0);
#pragma unroll
    for (int j = 0; j < NJ; ++j) { q[j] = q0[j]; qd[j] = qd0[j]; du[j] = R(0); }
    const int ext = Cc.ext_mode == EXTW_WALL ? EXTW_WALL : EXTW_NONE;
    for (int t = 0; t < T; ++t) {
        const ModelM<R>& M = *per_step(&Mc);
        const CostM<R>& C = *per_step(&Cc);
        R z[8], v[NJ], tau[NJ];
        normals8<R>(seed, tick, k, (uint32_t)t, z);
        noise_step(C, z, du, t);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            if (noise_out) noise_out[(size_t)(t * NJ + j) * noise_stride] = du[j];
            if (noise_lds) noise_lds[(t * NJ + j) * lds_stride] = du[j];
            v[j] = R(U_nom[t * NJ + j]) + du[j];
            tau[j] = v[j] + tau_ext_c[j];
        }
        StepOut<R> o;
        if constexpr (EXPLICIT) dyn_step_m<R, FORCE>(M, C, ext, q, qd, tau, v, o);
        else dyn_step<R, FORCE>(M, C, ext, q, qd, tau, v, o);
        R l = motion_cost(M, C, tg, o.pee, o.Rn) + joint_cost(M, C, q, qd) + torque_cost(M, C, v);
        if (FORCE) l += force_cost(C, tg, o.F);
        if constexpr (COLL) l += collision_cost(M, C, q);   // Eq. 14's C_collision
        S += l;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            qd[j] += o.qdd[j] * C.dt;
            q[j] += qd[j] * C.dt;
        }
    }
    R pee[3], Rn[9];
    fk_ee(Mc, q, pee, Rn, (R*)nullptr, (R*)nullptr);
    S += Cc.w_T * (motion_cost(Mc, Cc, tg, pee, Rn) + joint_cost(Mc, Cc, q, qd));
    return S;
}

}  // namespace mppi
