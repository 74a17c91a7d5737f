// model_prep.hpp -- converts the C-ABI robot/cost structs into the layout the
// rollout kernels read (ModelM / CostM): a field copy with a cast to the
// rollout precision (run on the device for the model, on the host for the
// cost).
#pragma once

#include <cmath>

#include "dyn.hpp"
#include "mppi.h"

namespace mppi {

template <typename R> MPPI_HD void prep_link(const mppi_link_params& P, LinkM<R>& L)
{
    for (int a = 0; a < 9; ++a) L.Rp[a] = R(P.R_parent[a]);
    for (int a = 0; a < 3; ++a) L.rp[a] = R(P.r_parent[a]);
    const double m = P.mass;
    for (int a = 0; a < 6; ++a) L.Ic[a] = R(P.inertia_com[a]);
    for (int a = 0; a < 3; ++a) L.com[a] = R(P.com[a]);
    L.m = R(m);
    L.arm = R(P.armature);
    L.qmin = R(P.q_min); L.qmax = R(P.q_max); L.qdmax = R(P.qd_max); L.taumax = R(P.tau_max);
}

template <typename R> MPPI_HD void prep_model(const mppi_robot_params& P, ModelM<R>& M)
{
    for (int i = 0; i < NJ; ++i) prep_link(P.link[i], M.L[i]);
    for (int a = 0; a < 9; ++a) M.Ree[a] = R(P.R_ee[a]);
    for (int a = 0; a < 3; ++a) { M.ree[a] = R(P.r_ee[a]); M.g[a] = R(P.gravity[a]); }
}

static_assert(MPPI_MAX_OBSTACLES == 4 && MPPI_MAX_PAIRS == 32, "CostM collision arrays");

template <typename R> inline void prep_cost(const mppi_cost_params& P, CostM<R>& C)
{
    C.dt = R(P.dt);
    int ori = 0, force = 0;
    for (int j = 0; j < NJ; ++j) { C.sigma[j] = R(P.sigma[j]); C.q_rest[j] = R(P.q_rest[j]); }
    C.rho = R(P.noise_rho);
    const double rc = std::sqrt(1.0 - P.noise_rho * P.noise_rho);
    for (int j = 0; j < NJ; ++j) C.sig_c[j] = R(rc * P.sigma[j]);
    for (int a = 0; a < 3; ++a) {
        C.W_pos[a] = R(P.W_pos[a]); C.W_ori[a] = R(P.W_ori[a]);
        C.wall_n[a] = R(P.wall_n[a]);
        ori |= P.W_ori[a] != 0.0;
    }
    for (int a = 0; a < 6; ++a) {
        C.W_force[a] = R(P.W_force[a]); C.W_reg[a] = R(P.W_reg[a]); C.F_ext[a] = R(P.F_ext[a]);
        force |= (P.W_force[a] != 0.0) | (P.W_reg[a] != 0.0);
    }
    C.w_q = R(P.w_q); C.w_qd = R(P.w_qd); C.w_tau = R(P.w_tau); C.w_post = R(P.w_post);
    C.w_T = R(P.w_terminal);
    C.wall_d0 = R(P.wall_d0); C.wall_k = R(P.wall_k); C.wall_c = R(P.wall_c);
    C.ext_mode = P.ext_mode;
    C.force_mode = P.force_mode;
    C.has_ori = ori;
    C.has_force = force;
    C.w_coll = R(P.w_collision);
    for (int o = 0; o < 4; ++o)
        for (int a = 0; a < 6; ++a) C.obs[o][a] = o < P.n_obstacles ? R(P.obstacles[o][a]) : R(0);
    C.n_pairs = P.n_pairs;
    for (int i = 0; i < 32; ++i) {
        const bool on = i < P.n_pairs;
        C.pa[i] = on ? P.pairs[i][0] : 0;
        C.pb[i] = on ? P.pairs[i][1] : 0;
        C.dth2[i] = on ? R(P.d_th[i]) * R(P.d_th[i]) : R(0);
    }
}

}  // namespace mppi
