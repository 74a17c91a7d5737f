// Counts the floating-point operations of the rollout kernels' per-sample
// math (dyn.hpp / rollout.hpp) by instantiating it on the host with an
// op-counting scalar.  add/sub, mul, div, sqrt count 1 flop each (a fused
// multiply-add is a mul plus an add); sin/cos/log/exp/atan2 are counted
// separately.  Integer Philox arithmetic is not counted.
#include <cmath>
#include <cstdint>
#include <cstring>

namespace mppi {
struct Flop;
}

#include "mppi.h"

namespace mppi {
struct Counts {
    long long add = 0, mul = 0, div = 0, sqrt = 0, trans = 0, cmp = 0;
};
static Counts g_counts;

struct Flop {
    double v;
    Flop() : v(0) {}
    Flop(double x) : v(x) {}
    Flop(float x) : v(x) {}
    Flop(int x) : v(x) {}
    Flop(unsigned x) : v(x) {}
    explicit operator double() const { return v; }
};
inline Flop operator+(Flop a, Flop b) { g_counts.add++; return Flop(a.v + b.v); }
inline Flop operator-(Flop a, Flop b) { g_counts.add++; return Flop(a.v - b.v); }
inline Flop operator*(Flop a, Flop b) { g_counts.mul++; return Flop(a.v * b.v); }
inline Flop operator/(Flop a, Flop b) { g_counts.div++; return Flop(a.v / b.v); }
inline Flop operator-(Flop a) { return Flop(-a.v); }
inline Flop& operator+=(Flop& a, Flop b) { a = a + b; return a; }
inline Flop& operator-=(Flop& a, Flop b) { a = a - b; return a; }
inline Flop& operator*=(Flop& a, Flop b) { a = a * b; return a; }
inline bool operator<(Flop a, Flop b) { g_counts.cmp++; return a.v < b.v; }
inline bool operator>(Flop a, Flop b) { g_counts.cmp++; return a.v > b.v; }
inline bool operator>=(Flop a, Flop b) { g_counts.cmp++; return a.v >= b.v; }
inline bool operator<=(Flop a, Flop b) { g_counts.cmp++; return a.v <= b.v; }
inline bool operator==(Flop a, Flop b) { g_counts.cmp++; return a.v == b.v; }
inline void sincos_(Flop x, Flop* s, Flop* c) { g_counts.trans += 2; *s = Flop(std::sin(x.v)); *c = Flop(std::cos(x.v)); }
inline void sincospi_(Flop x, Flop* s, Flop* c)
{
    g_counts.trans += 2;
    *s = Flop(std::sin(M_PI * x.v));
    *c = Flop(std::cos(M_PI * x.v));
}
inline Flop sqrt_(Flop x) { g_counts.sqrt++; return Flop(std::sqrt(x.v)); }
inline Flop log_(Flop x) { g_counts.trans++; return Flop(std::log(x.v)); }
inline Flop atan2_(Flop y, Flop x) { g_counts.trans++; return Flop(std::atan2(y.v, x.v)); }
inline Flop abs_(Flop x) { return Flop(std::fabs(x.v)); }
inline Flop fma_(Flop a, Flop b, Flop c) { g_counts.mul++; g_counts.add++; return Flop(a.v * b.v + c.v); }
inline Flop rcp_(Flop x) { g_counts.div++; return Flop(1.0 / x.v); }
inline Flop rsqrt_sqrt_(Flop x) { g_counts.sqrt++; return Flop(std::sqrt(x.v)); }
inline Flop max0_(Flop x) { g_counts.cmp++; return Flop(x.v > 0 ? x.v : 0.0); }
}  // namespace mppi

#include "model_prep.hpp"
#include "rollout.hpp"

using namespace mppi;

// counts[6] = add, mul, div, sqrt, trans, cmp for one rollout of T steps
extern "C" void oc_rollout(const mppi_robot_params* rp, const mppi_cost_params* cp, const double* target,
                           const double* q0, const double* qd0, const double* U, int T, long long* counts)
{
    ModelM<Flop> M;
    CostM<Flop> C;
    TargetM<Flop> tg;
    prep_model(*rp, M);
    prep_cost(*cp, C);
    make_target(target, tg);
    Flop q[NJ], qd[NJ], te[NJ];
    for (int j = 0; j < NJ; ++j) { q[j] = Flop(q0[j]); qd[j] = Flop(qd0[j]); te[j] = Flop(0.0); }
    Flop nz[256 * NJ];
    g_counts = Counts();
    const bool ex = cp->dynamics == MPPI_DYN_EXPLICIT_M;
    // (the collision term is counted only when enabled; its per-pair work
    // depends on the clamping branch taken)
    if (cp->n_pairs > 0) {
        if (C.has_force) rollout_sample<Flop, true, false, true>(M, C, tg, q, qd, te, U, T, 1, 0, 0, nz, 1);
        else rollout_sample<Flop, false, false, true>(M, C, tg, q, qd, te, U, T, 1, 0, 0, nz, 1);
    } else if (C.has_force) {
        if (ex) rollout_sample<Flop, true, true>(M, C, tg, q, qd, te, U, T, 1, 0, 0, nz, 1);
        else rollout_sample<Flop, true>(M, C, tg, q, qd, te, U, T, 1, 0, 0, nz, 1);
    } else {
        if (ex) rollout_sample<Flop, false, true>(M, C, tg, q, qd, te, U, T, 1, 0, 0, nz, 1);
        else rollout_sample<Flop, false>(M, C, tg, q, qd, te, U, T, 1, 0, 0, nz, 1);
    }
    counts[0] = g_counts.add; counts[1] = g_counts.mul; counts[2] = g_counts.div;
    counts[3] = g_counts.sqrt; counts[4] = g_counts.trans; counts[5] = g_counts.cmp;
}
