"""GPU parity of the eight-lanes-per-sample update (mppi_set_launch(h, 8):
one lane per joint and one for the EE frame; composite-rigid-body inertia
and an LDL^T solve instead of the articulated-body recursion) against the
FP64 oracle, with the criteria of the other parity tests: per-sample cost
relative error <= 1e-4 (conditioning allowance for the force estimate),
noise equal to the oracle's to FP32 rounding, U_new within 1e-3 N m
(stage-isolated always, end-to-end when the cost errors cannot move the
weights)."""
import numpy as np
import pytest

from paper_2609_02020_amd import binding as B
from gpu_util import (KAPPA_CAP, U32, U_ATOL, check_costs_fp32, check_update, cost_rel_err, device_update,
                      force_condition)

pytestmark = pytest.mark.gpu
GROUP = 8
K_FLAG_MAX = 20


def oracle_update(ora, case, cost, seed, tick):
    st, U, S, E = ora.update(case["robot"], cost, case["target"], case["q0"], case["qd0"],
                             case["U_nom"], seed, tick)
    assert st == 0
    return U, S, E


def resized(base, K, T, **extra):
    U = np.asarray(base["U_nom"])
    U = np.concatenate([U] * (T // len(U) + 1))[:T]
    cost = dict(base["cost"], K=K, T=T, **extra)
    return dict(base, cost=cost, U_nom=U.tolist())


def group_update(case, seed, tick, **solver_kw):
    solver = B.Solver(case["robot"], case["cost"], B.FP32, **solver_kw)
    solver.set_launch(GROUP)
    out = device_update(solver, case, seed, tick, B.FP32)
    solver.close()
    return out


def test_group_full_size_contact_parity(ora, workloads):
    """K = 4096, T = 18, wall contact and force cost: every sample."""
    for i, case in enumerate(workloads["wall_k4096"][:2]):
        print("case wall_k4096[%d], eight lanes per sample" % i, flush=True)
        out = group_update(case, case["seed"], 7)
        U_ref, S_ref, E_ref = oracle_update(ora, case, case["cost"], case["seed"], 7)
        assert out["status"] == B.OK
        err = cost_rel_err(out["costs"], S_ref)
        print("max cost rel err %.3g, p99 %.3g, median %.3g" % (err.max(), np.percentile(err, 99), np.median(err)))
        flagged = check_costs_fp32(ora, case, out["costs"], S_ref, case["seed"], 7, "group wall %d" % i)
        assert len(flagged) <= K_FLAG_MAX
        assert np.abs(out["noise"] - E_ref).max() <= 5e-5
        note = check_update(ora, case, out, case["cost"]["lambda"], S_ref, U_ref, "group wall %d" % i)
        if note:
            print(note)


@pytest.mark.parametrize("which,i,K,T,extra", [
    ("single_k256", 0, 256, 18, {}),
    ("single_k256", 1, 1, 18, {}),
    ("single_k256", 2, 31, 7, {}),
    ("wall_k4096", 3, 33, 1, {}),
    ("wall_k4096", 4, 1000, 5, {"noise_rho": 0.6}),
    ("wall_k4096", 5, 4097, 3, {}),
    ("wall_k4096", 6, 300, 40, {"force_mode": 1}),
    ("single_k256", 3, 500, 18, {"ext_mode": 1, "F_ext": [3.0, -2.0, 5.0, 0.2, -0.1, 0.3]}),
])
def test_group_ragged_sizes_and_variants(ora, workloads, which, i, K, T, extra):
    """Ragged K (partial groups and workgroups), short and long horizons,
    correlated noise, literal tau_F, the constant external wrench."""
    case = resized(workloads[which][i], K, T, **extra)
    print("%s[%d] K=%d T=%d %s" % (which, i, K, T, extra), flush=True)
    out = group_update(case, 99, 3)
    U_ref, S_ref, E_ref = oracle_update(ora, case, case["cost"], 99, 3)
    assert out["status"] == B.OK
    check_costs_fp32(ora, case, out["costs"], S_ref, 99, 3, "group ragged")
    assert np.abs(out["noise"] - E_ref).max() <= 5e-5
    note = check_update(ora, case, out, case["cost"]["lambda"], S_ref, U_ref, "group ragged")
    if note:
        print(note)
    if K == 1:   # one sample returns its own perturbation (Eq. 4b with one term)
        assert np.abs(out["U_new"] - (np.asarray(case["U_nom"]) + out["noise"][0])).max() < 1e-6
    assert np.array_equal(out["U_shift"][:-1], out["U_new"][1:])
    assert np.array_equal(out["U_shift"][-1], out["U_new"][-1])


@pytest.mark.parametrize("which,i", [("wall_k4096", 0), ("single_k256", 4)])
def test_group_matches_two_wave_update(ora, workloads, which, i):
    """The same update with the default two-wave launch: the noise is
    bitwise the same (the same Philox words and arithmetic per normal); the
    costs agree to FP32 rounding of two factorisations, except for samples
    whose force estimate inverts an ill-conditioned J M^-1 J^T, where both
    sides carry up to min(kappa u32, 1e-2) each; U_new agrees to 1e-3 N m."""
    case = workloads[which][i]
    outs = []
    for w in (2, GROUP):
        solver = B.Solver(case["robot"], case["cost"], B.FP32)
        solver.set_launch(w)
        outs.append(device_update(solver, case, case["seed"], 12, B.FP32))
        solver.close()
    two, grp = outs
    assert np.array_equal(two["noise"], grp["noise"])
    rel = cost_rel_err(grp["costs"], two["costs"])
    print("%s[%d]: max rel cost difference %.3g, p99 %.3g, median %.3g"
          % (which, i, rel.max(), np.percentile(rel, 99), np.median(rel)))
    assert np.median(rel) <= 1e-5
    flagged = []
    for k in np.nonzero(rel > 2e-4)[0]:
        kappa = force_condition(ora, case, case["seed"], 12, int(k))
        flagged.append((int(k), float(rel[k]), kappa))
        assert rel[k] <= min(2 * kappa * U32, 2 * KAPPA_CAP), (k, rel[k], kappa)
    print("ill-conditioned samples (k, rel difference, kappa):", flagged)
    assert len(flagged) <= K_FLAG_MAX
    assert np.abs(two["U_new"] - grp["U_new"]).max() <= U_ATOL


def test_group_small_lambda_fp64_weights(ora, workloads):
    """lambda = 0.01 (below the FP64 threshold): Eq. 4 accumulates in FP64
    inside the group kernel; stage-isolated U_new against the oracle's
    weighting of the GPU's own costs and noise."""
    case = workloads["wall_k4096"][7]
    case = dict(case, cost=dict(case["cost"], **{"lambda": 0.01}))
    out = group_update(case, case["seed"], 4)
    assert out["status"] == B.OK
    st, U_stage, _ = ora.weights_update(out["costs"], out["noise"], case["U_nom"], 0.01)
    assert st == 0 and np.abs(out["U_new"] - U_stage).max() <= U_ATOL


@pytest.mark.parametrize("K,T", [(16384, 6), (320, 256)])
def test_group_many_partials_and_maximum_horizon(ora, workloads, K, T):
    """512 workgroup partials merged by the last workgroup; the longest
    horizon (the partial sums its rows in chunks of steps)."""
    base = workloads["wall_k4096"][5] if T < 100 else workloads["single_k256"][7]
    extra = {} if T < 100 else {"dt": 0.002}
    case = resized(base, K, T, **extra)
    out = group_update(case, 7, 1)
    U_ref, S_ref, E_ref = oracle_update(ora, case, case["cost"], 7, 1)
    assert out["status"] == B.OK
    check_costs_fp32(ora, case, out["costs"], S_ref, 7, 1, "group K=%d T=%d" % (K, T))
    assert np.abs(out["noise"] - E_ref).max() <= 5e-5
    note = check_update(ora, case, out, case["cost"]["lambda"], S_ref, U_ref, "group K=%d T=%d" % (K, T))
    if note:
        print(note)


def test_group_every_cost_non_finite(workloads):
    """Nominal torques of 1e30 N m: MPPI_ENONFINITE and the nominal sequence
    passed through, its shift included."""
    case = workloads["wall_k4096"][2]
    cost = dict(case["cost"], K=1000)
    U = np.full((cost["T"], 7), 1e30)
    solver = B.Solver(case["robot"], cost, B.FP32)
    solver.set_launch(GROUP)
    out = device_update(solver, dict(case, cost=cost), case["seed"], 1, B.FP32, U_nom=U)
    solver.close()
    assert out["status"] == B.ENONFINITE
    assert not np.isfinite(out["costs"]).any()
    assert np.array_equal(out["U_new"], U)
    assert np.array_equal(out["U_shift"][:-1], U[1:]) and np.array_equal(out["U_shift"][-1], U[-1])
