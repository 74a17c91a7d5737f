// Host-only build of the rollout kernels' per-sample math (dyn.hpp,
// rollout.hpp, model_prep.hpp), for CPU unit tests against the oracle and
// for counting the algorithmic floating-point work of one sample-step.
// Never loaded by the product library.
#include <cmath>
#include <cstdint>
#include <cstring>

#include "mppi.h"
#include "model_prep.hpp"
#include "rollout.hpp"

using namespace mppi;

template <typename R, bool EXPLICIT = false>
static void step_t(const mppi_robot_params* rp, const mppi_cost_params* cp, int force, int ext,
                   const double* q, const double* qd, const double* tau, const double* v,
                   double* qdd, double* pee, double* Rn, double* F)
{
    ModelM<R> M;
    CostM<R> C;
    prep_model(*rp, M);
    prep_cost(*cp, C);
    R qq[NJ], qqd[NJ], tt[NJ], vv[NJ];
    for (int j = 0; j < NJ; ++j) { qq[j] = R(q[j]); qqd[j] = R(qd[j]); tt[j] = R(tau[j]); vv[j] = R(v[j]); }
    StepOut<R> o;
    if (EXPLICIT) {
        if (force) dyn_step_m<R, true>(M, C, ext, qq, qqd, tt, vv, o);
        else dyn_step_m<R, false>(M, C, ext, qq, qqd, tt, vv, o);
    } else {
        if (force) dyn_step<R, true>(M, C, ext, qq, qqd, tt, vv, o);
        else dyn_step<R, false>(M, C, ext, qq, qqd, tt, vv, o);
    }
    for (int j = 0; j < NJ; ++j) qdd[j] = double(o.qdd[j]);
    for (int a = 0; a < 3; ++a) pee[a] = double(o.pee[a]);
    for (int a = 0; a < 9; ++a) Rn[a] = double(o.Rn[a]);
    if (force) for (int a = 0; a < 6; ++a) F[a] = double(o.F[a]);
}

extern "C" void hc_step(const mppi_robot_params* rp, const mppi_cost_params* cp, int prec, int force,
                        int ext, const double* q, const double* qd, const double* tau,
                        const double* v, double* qdd, double* pee, double* Rn, double* F)
{
    const bool ex = cp->dynamics == MPPI_DYN_EXPLICIT_M;
    if (prec == MPPI_FP64) {
        if (ex) step_t<double, true>(rp, cp, force, ext, q, qd, tau, v, qdd, pee, Rn, F);
        else step_t<double>(rp, cp, force, ext, q, qd, tau, v, qdd, pee, Rn, F);
    } else {
        if (ex) step_t<float, true>(rp, cp, force, ext, q, qd, tau, v, qdd, pee, Rn, F);
        else step_t<float>(rp, cp, force, ext, q, qd, tau, v, qdd, pee, Rn, F);
    }
}

// The force-cost step with its force-estimate inputs handed over through a
// flat buffer (stride 3, as the two-wave update hands them over through
// LDS) and the estimate formed from the buffer: F_split.  The same step's
// inline estimate goes to F; qdd must be the same in both runs.
extern "C" void hc_step_handoff(const mppi_robot_params* rp, const mppi_cost_params* cp, const double* q,
                                const double* qd, const double* tau, const double* v, double* F,
                                double* F_split, double* qdd_diff)
{
    ModelM<double> M;
    CostM<double> C;
    prep_model(*rp, M);
    prep_cost(*cp, C);
    const int ext = C.ext_mode == EXTW_WALL ? EXTW_WALL : EXTW_NONE;
    StepOut<double> a, b;
    dyn_step<double, true>(M, C, ext, q, qd, tau, v, a);
    double buf[kFiCount * 3];
    for (int i = 0; i < kFiCount * 3; ++i) buf[i] = NAN;
    dyn_step<double, true>(M, C, ext, q, qd, tau, v, b, buf, 3);
    ForceIn<double> fi;
    for (int i = 0; i < NJ; ++i) {
        for (int c = 0; c < 3; ++c) {
            fi.z[i][c] = buf[(kFiZ + 3 * i + c) * 3];
            fi.rr[i][c] = buf[(kFiRr + 3 * i + c) * 3];
        }
        for (int c = 0; c < 6; ++c) fi.U[i][c] = buf[(kFiU + 6 * i + c) * 3];
        fi.iD[i] = buf[(kFiD + i) * 3];
    }
    for (int c = 0; c < 3; ++c) fi.ree[c] = buf[(kFiRee + c) * 3];
    force_estimate(fi, v, M.g, C.force_mode, F_split);
    for (int c = 0; c < 6; ++c) F[c] = a.F[c];
    double d = 0.0;
    for (int j = 0; j < NJ; ++j) d = std::fmax(d, std::fabs(a.qdd[j] - b.qdd[j]));
    *qdd_diff = d;
}

template <typename R>
static double rollout_t(const mppi_robot_params* rp, const mppi_cost_params* cp, const double* target,
                        const double* q0, const double* qd0, const double* U, uint64_t seed,
                        uint64_t tick, uint32_t k, double* noise)
{
    ModelM<R> M;
    CostM<R> C;
    TargetM<R> tg;
    prep_model(*rp, M);
    prep_cost(*cp, C);
    make_target(target, tg);
    R q[NJ], qd[NJ], te[NJ] = {};
    for (int j = 0; j < NJ; ++j) { q[j] = R(q0[j]); qd[j] = R(qd0[j]); }
    if (C.ext_mode == EXTW_CONST) const_ext_torque(M, C, q, te);
    R nz[256 * NJ];
    const bool ex = cp->dynamics == MPPI_DYN_EXPLICIT_M, co = cp->n_pairs > 0;
    const uint32_t tk = (uint32_t)tick;
    R S;
    if (co)
        S = C.has_force ? (ex ? rollout_sample<R, true, true, true>(M, C, tg, q, qd, te, U, cp->T, seed, tk, k, nz, 1)
                              : rollout_sample<R, true, false, true>(M, C, tg, q, qd, te, U, cp->T, seed, tk, k, nz, 1))
                        : (ex ? rollout_sample<R, false, true, true>(M, C, tg, q, qd, te, U, cp->T, seed, tk, k, nz, 1)
                              : rollout_sample<R, false, false, true>(M, C, tg, q, qd, te, U, cp->T, seed, tk, k, nz, 1));
    else
        S = C.has_force ? (ex ? rollout_sample<R, true, true>(M, C, tg, q, qd, te, U, cp->T, seed, tk, k, nz, 1)
                              : rollout_sample<R, true>(M, C, tg, q, qd, te, U, cp->T, seed, tk, k, nz, 1))
                        : (ex ? rollout_sample<R, false, true>(M, C, tg, q, qd, te, U, cp->T, seed, tk, k, nz, 1)
                              : rollout_sample<R, false>(M, C, tg, q, qd, te, U, cp->T, seed, tk, k, nz, 1));
    for (int i = 0; i < cp->T * NJ; ++i) noise[i] = double(nz[i]);
    return double(S);
}

extern "C" double hc_rollout(const mppi_robot_params* rp, const mppi_cost_params* cp, int prec,
                             const double* target, const double* q0, const double* qd0,
                             const double* U, uint64_t seed, uint64_t tick, uint32_t k,
                             double* noise)
{
    if (prec == MPPI_FP64) return rollout_t<double>(rp, cp, target, q0, qd0, U, seed, tick, k, noise);
    return rollout_t<float>(rp, cp, target, q0, qd0, U, seed, tick, k, noise);
}

extern "C" void hc_normals(int prec, uint64_t seed, uint64_t tick, uint32_t k, uint32_t t, double* z)
{
    if (prec == MPPI_FP64) {
        double zz[8];
        normals8<double>(seed, (uint32_t)tick, k, t, zz);
        for (int i = 0; i < 8; ++i) z[i] = zz[i];
    } else {
        float zz[8];
        normals8<float>(seed, (uint32_t)tick, k, t, zz);
        for (int i = 0; i < 8; ++i) z[i] = zz[i];
    }
}

extern "C" double hc_seg_dist2(int prec, const double* a0, const double* a1, const double* b0, const double* b1)
{
    if (prec == MPPI_FP64) return seg_dist2<double>(a0, a1, b0, b1);
    float f[4][3];
    for (int c = 0; c < 3; ++c) { f[0][c] = float(a0[c]); f[1][c] = float(a1[c]); f[2][c] = float(b0[c]); f[3][c] = float(b1[c]); }
    return double(seg_dist2<float>(f[0], f[1], f[2], f[3]));
}

template <typename R>
static double collision_t(const mppi_robot_params* rp, const mppi_cost_params* cp, const double* q)
{
    ModelM<R> M;
    CostM<R> C;
    prep_model(*rp, M);
    prep_cost(*cp, C);
    R qq[NJ];
    for (int j = 0; j < NJ; ++j) qq[j] = R(q[j]);
    return double(collision_cost(M, C, qq));
}

extern "C" double hc_collision(const mppi_robot_params* rp, const mppi_cost_params* cp, int prec, const double* q)
{
    return prec == MPPI_FP64 ? collision_t<double>(rp, cp, q) : collision_t<float>(rp, cp, q);
}

// ---------------------------------------------------------------------------
// The eight-lane group rollout (group.hpp) on the host: eight threads run
// the per-lane code and meet at every cross-lane move, which is what the
// lanes of one group do in lockstep on the device.
// ---------------------------------------------------------------------------
#include <condition_variable>
#include <mutex>
#include <thread>
#include <vector>

#include "group.hpp"

struct HostGroupSync {
    std::mutex mu;
    std::condition_variable cv;
    int count = 0;
    long phase = 0;
    double slot[kGroup];
    void barrier()
    {
        std::unique_lock<std::mutex> lk(mu);
        const long ph = phase;
        if (++count == kGroup) {
            count = 0;
            ++phase;
            cv.notify_all();
        } else {
            cv.wait(lk, [&] { return phase != ph; });
        }
    }
};

template <typename R> struct HostGroup {
    int j;
    HostGroupSync* s;
    R* shm;
    template <int D> R shr(R x) const
    {
        s->slot[j] = double(x);
        s->barrier();
        const R r = j >= D ? R(s->slot[j - D]) : R(0);
        s->barrier();
        return r;
    }
    template <int D> R shr_one(R x) const
    {
        s->slot[j] = double(x);
        s->barrier();
        const R r = j >= D ? R(s->slot[j - D]) : R(1);
        s->barrier();
        return r;
    }
    template <int D> R add_shr(R x) const { return x + shr<D>(x); }
    template <int D> R add_shl(R x) const
    {
        s->slot[j] = double(x);
        s->barrier();
        const R r = j + D < kGroup ? R(s->slot[j + D]) : R(0);
        s->barrier();
        return x + r;
    }
    template <int K> R bcast(R x) const
    {
        s->slot[j] = double(x);
        s->barrier();
        const R r = R(s->slot[K]);
        s->barrier();
        return r;
    }
    // the device's butterfly: x + x^1, then + ^2, then + ^4
    R sum(R x) const
    {
        s->slot[j] = double(x);
        s->barrier();
        R a[kGroup], b[kGroup];
        for (int i = 0; i < kGroup; ++i) a[i] = R(s->slot[i]) + R(s->slot[i ^ 1]);
        for (int i = 0; i < kGroup; ++i) b[i] = a[i] + a[i ^ 2];
        const R r = b[j] + b[j ^ 4];
        s->barrier();
        return r;
    }
    void sync() const { s->barrier(); }
};

template <typename R, typename F> static void run_group(F&& body)
{
    HostGroupSync sy;
    std::vector<R> shm(kGxCount, R(NAN));
    std::thread th[kGroup];
    for (int j = 0; j < kGroup; ++j) {
        th[j] = std::thread([&, j] {
            HostGroup<R> g{j, &sy, shm.data()};
            body(g);
        });
    }
    for (auto& t : th) t.join();
}

template <typename R>
static void group_step_t(const mppi_robot_params* rp, const mppi_cost_params* cp, int force, int ext,
                         const double* q, const double* qd, const double* tau, const double* v,
                         double* qdd, double* pee, double* Re, double* F)
{
    ModelM<R> M;
    CostM<R> C;
    prep_model(*rp, M);
    prep_cost(*cp, C);
    TargetM<R> tg;
    const double tgt[13] = {0, 0, 0, 1, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    make_target(tgt, tg);
    GroupStepOut<R> out[kGroup];
    run_group<R>([&](const HostGroup<R>& g) {
        GroupLink<R> L;
        group_link(M, C, g.j, L);
        const int jc = g.j < NJ ? g.j : NJ - 1;
        const R qj = g.j < NJ ? R(q[jc]) : R(0), qdj = g.j < NJ ? R(qd[jc]) : R(0);
        const R tj = g.j < NJ ? R(tau[jc]) : R(0), vj = g.j < NJ ? R(v[jc]) : R(0);
        R a;
        if (force) group_step<R, true>(g, L, C, tg, M.g, ext, qj, qdj, tj, vj, a, &out[g.j]);
        else group_step<R, false>(g, L, C, tg, M.g, ext, qj, qdj, tj, vj, a, &out[g.j]);
    });
    for (int j = 0; j < NJ; ++j) qdd[j] = double(out[j].qdd);
    for (int a = 0; a < 3; ++a) pee[a] = double(out[NJ].pee[a]);
    for (int a = 0; a < 9; ++a) Re[a] = double(out[NJ].Re[a]);
    for (int a = 0; a < 6; ++a) F[a] = double(out[force ? 0 : NJ].F[a]);
}

// One step on the group: qdd[7], the EE point, R_ee (EE frame, not the
// last link's) and the force estimate (from lane 0, force != 0).
extern "C" void hc_group_step(const mppi_robot_params* rp, const mppi_cost_params* cp, int prec, int force,
                              int ext, const double* q, const double* qd, const double* tau, const double* v,
                              double* qdd, double* pee, double* Re, double* F)
{
    if (prec == MPPI_FP64) group_step_t<double>(rp, cp, force, ext, q, qd, tau, v, qdd, pee, Re, F);
    else group_step_t<float>(rp, cp, force, ext, q, qd, tau, v, qdd, pee, Re, F);
}

template <typename R>
static double group_rollout_t(const mppi_robot_params* rp, const mppi_cost_params* cp, const double* target,
                              const double* q0, const double* qd0, const double* U, uint64_t seed,
                              uint64_t tick, uint32_t k, double* noise, bool split = false)
{
    ModelM<R> M;
    CostM<R> C;
    TargetM<R> tg;
    prep_model(*rp, M);
    prep_cost(*cp, C);
    make_target(target, tg);
    R q[NJ], qd[NJ], te[NJ] = {};
    for (int j = 0; j < NJ; ++j) { q[j] = R(q0[j]); qd[j] = R(qd0[j]); }
    if (C.ext_mode == EXTW_CONST) const_ext_torque(M, C, q, te);
    const int T = cp->T;
    std::vector<R> nz((size_t)T * NJ, R(0));
    R S[kGroup];
    run_group<R>([&](const HostGroup<R>& g) {
        GroupLink<R> L;
        group_link(M, C, g.j, L);
        const bool live = g.j < NJ;
        const int jc = live ? g.j : NJ - 1;
        const R qj = live ? q[jc] : R(0), qdj = live ? qd[jc] : R(0), tj = live ? te[jc] : R(0);
        using HG = HostGroup<R>;
        const uint32_t tk = (uint32_t)tick;
        if (cp->n_pairs > 0)
            S[g.j] = C.has_force
                         ? group_rollout<R, true, HG, double, true>(g, L, C, tg, M.g, qj, qdj, tj, U, T, seed, tk, k,
                                                                    nz.data(), 1, nullptr, 0, split)
                         : group_rollout<R, false, HG, double, true>(g, L, C, tg, M.g, qj, qdj, tj, U, T, seed, tk, k,
                                                                     nz.data(), 1, nullptr, 0, split);
        else
            S[g.j] = C.has_force
                         ? group_rollout<R, true>(g, L, C, tg, M.g, qj, qdj, tj, U, T, seed, tk, k, nz.data(), 1,
                                                  nullptr, 0, split)
                         : group_rollout<R, false>(g, L, C, tg, M.g, qj, qdj, tj, U, T, seed, tk, k, nz.data(), 1,
                                                   nullptr, 0, split);
    });
    for (int i = 0; i < T * NJ; ++i) noise[i] = double(nz[i]);
    for (int j = 1; j < kGroup; ++j)
        if (!(S[j] == S[0])) return NAN;   // every lane must hold the same total
    return double(S[0]);
}

extern "C" double hc_group_rollout(const mppi_robot_params* rp, const mppi_cost_params* cp, int prec,
                                   const double* target, const double* q0, const double* qd0, const double* U,
                                   uint64_t seed, uint64_t tick, uint32_t k, double* noise)
{
    if (prec == MPPI_FP64) return group_rollout_t<double>(rp, cp, target, q0, qd0, U, seed, tick, k, noise);
    return group_rollout_t<float>(rp, cp, target, q0, qd0, U, seed, tick, k, noise);
}

// The same rollout with each step split into its dynamics and cost parts,
// as the eight-lane batch kernel runs it (the factor of M handed over
// through the group area).
extern "C" double hc_group_rollout_split(const mppi_robot_params* rp, const mppi_cost_params* cp, int prec,
                                         const double* target, const double* q0, const double* qd0,
                                         const double* U, uint64_t seed, uint64_t tick, uint32_t k, double* noise)
{
    if (prec == MPPI_FP64) return group_rollout_t<double>(rp, cp, target, q0, qd0, U, seed, tick, k, noise, true);
    return group_rollout_t<float>(rp, cp, target, q0, qd0, U, seed, tick, k, noise, true);
}
