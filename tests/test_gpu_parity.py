"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle
on the same seeded inputs and the same Philox counters.

Criteria: per-sample cost relative error <= 1e-4; U_new within 1e-3 N m
(stage-isolated always; end-to-end when max |dS| / lambda <= 1e-3); noise
equal to the oracle's to FP32 rounding; integer-valued outcomes (status,
argmin selection) exact.
"""
import numpy as np
import pytest

from paper_2609_02020_amd import binding as B
from gpu_util import (COST_RTOL, U_ATOL, check_costs_fp32, check_update, cost_rel_err,
                      device_update, torch_dev)

pytestmark = pytest.mark.gpu
K_FLAG_MAX = 20   # at most this many of 4096 samples may need the conditioning allowance


def oracle_update(ora, case, cost, seed, tick):
    st, U, S, E = ora.update(case["robot"], cost, case["target"], case["q0"], case["qd0"],
                             case["U_nom"], seed, tick)
    assert st == 0
    return U, S, E


@pytest.mark.parametrize("precision", [B.FP64, B.FP32])
def test_single_update_k256_parity(ora, workloads, precision):
    notes = []
    for i, case in enumerate(workloads["single_k256"][:8]):
        print("case single_k256[%d] precision %d" % (i, precision), flush=True)
        solver = B.Solver(case["robot"], case["cost"], precision)
        out = device_update(solver, case, case["seed"], 0, precision)
        U_ref, S_ref, E_ref = oracle_update(ora, case, case["cost"], case["seed"], 0)
        rtol = 1e-9 if precision == B.FP64 else COST_RTOL
        assert cost_rel_err(out["costs"], S_ref).max() <= rtol
        assert np.abs(out["noise"] - E_ref).max() <= (1e-12 if precision == B.FP64 else 5e-5)
        assert out["status"] == B.OK
        note = check_update(ora, case, out, case["cost"]["lambda"], S_ref, U_ref, "case %d" % i)
        if note:
            notes.append(note)
        # the greedy limit selects the same sample (lambda = 1 and cost gaps >> 1)
        assert np.argmin(out["costs"]) == np.argmin(S_ref)
        solver.close()
    if precision == B.FP64:
        assert not notes
    print("\n".join(notes))


@pytest.mark.parametrize("launch", [8, 2, 1])
@pytest.mark.parametrize("tick", [7, 12])
def test_wall_k4096_full_size_parity(ora, workloads, launch, tick):
    """The K=4096, T=18 contact workload at full size, FP32, every sample,
    on each launch shape: eight lanes per sample (the default), two waves
    and one wave per 64 samples (the per-lane articulated-body kernels)."""
    for i, case in enumerate(workloads["wall_k4096"][:2]):
        print("case wall_k4096[%d] launch %d tick %d" % (i, launch, tick), flush=True)
        solver = B.Solver(case["robot"], case["cost"], B.FP32)
        solver.set_launch(launch)
        out = device_update(solver, case, case["seed"], tick, B.FP32)
        U_ref, S_ref, E_ref = oracle_update(ora, case, case["cost"], case["seed"], tick)
        err = cost_rel_err(out["costs"], S_ref)
        print("max cost rel err %.3g, p99 %.3g, median %.3g" % (err.max(), np.percentile(err, 99),
                                                               np.median(err)))
        flagged = check_costs_fp32(ora, case, out["costs"], S_ref, case["seed"], tick,
                                   "wall %d launch %d" % (i, launch))
        assert len(flagged) <= K_FLAG_MAX
        assert np.percentile(err, 99) <= 3e-6
        assert np.abs(out["noise"] - E_ref).max() <= 5e-5
        note = check_update(ora, case, out, 1.0, S_ref, U_ref, "wall %d" % i)
        if note:
            print(note)
        solver.close()


@pytest.mark.parametrize("K,T", [(1, 18), (63, 7), (65, 1), (1000, 5), (4097, 3), (300, 40)])
def test_ragged_sizes(ora, workloads, K, T):
    case = workloads["wall_k4096"][3]
    cost = dict(case["cost"], K=K, T=T)
    U = np.array(case["U_nom"])
    case = dict(case, cost=cost, U_nom=np.concatenate([U, np.repeat(U[-1:], max(0, T - len(U)), 0)])[:T])
    print("ragged K=%d T=%d" % (K, T), flush=True)
    solver = B.Solver(case["robot"], cost, B.FP32)
    out = device_update(solver, case, 99, 3, B.FP32)
    U_ref, S_ref, E_ref = oracle_update(ora, case, cost, 99, 3)
    check_costs_fp32(ora, case, out["costs"], S_ref, 99, 3, "ragged")
    check_update(ora, case, out, 1.0, S_ref, U_ref, "ragged")
    if K == 1:  # a single sample returns its own noise (Eq. 4b with one term)
        assert np.abs(out["U_new"] - (case["U_nom"] + out["noise"][0])).max() < 1e-6
    # the warm start is U_new shifted by one step, last row repeated
    assert np.array_equal(out["U_shift"][:-1], out["U_new"][1:])
    assert np.array_equal(out["U_shift"][-1], out["U_new"][-1])
    solver.close()


def test_weights_stage_non_finite_and_small_lambda(ora, workloads):
    torch, dev = torch_dev()
    case = workloads["single_k256"][1]
    K, T = 256, 18
    rng = np.random.default_rng(4)
    S = rng.uniform(100, 200, K)
    S[[3, 50, 200]] = [np.nan, np.inf, -np.inf]
    E = rng.normal(size=(K, T, 7)) * 2
    noise_dev = torch.tensor(E.transpose(1, 2, 0).reshape(-1).copy(), dtype=torch.float32, device=dev)
    for lam, thr in [(1.0, 0.05), (5.0, 0.05), (1e-6, 0.05), (1e-6, 0.0)]:
        cost = dict(case["cost"], **{"lambda": lam})
        solver = B.Solver(case["robot"], cost, B.FP32, lambda_fp64_threshold=thr)
        costs_dev = torch.tensor(S, dtype=torch.float32, device=dev)
        out = device_update(solver, case, 0, 0, B.FP32, stage=True, costs_in=costs_dev,
                            noise_in=noise_dev)
        S32 = S.astype(np.float32).astype(np.float64)
        E32 = E.astype(np.float32).astype(np.float64)
        st, U_ref, w = ora.weights_update(S32, E32, case["U_nom"], lam)
        assert out["status"] == B.OK
        tol = 1e-5 if lam >= 1e-3 else 1e-6
        assert np.abs(out["U_new"] - U_ref).max() <= tol, (lam, thr)
        solver.close()
    # every cost non-finite: status ENONFINITE and the nominal sequence back
    solver = B.Solver(case["robot"], case["cost"], B.FP32)
    bad = torch.tensor(np.full(K, np.nan), dtype=torch.float32, device=dev)
    out = device_update(solver, case, 0, 0, B.FP32, stage=True, costs_in=bad, noise_in=noise_dev)
    assert out["status"] == B.ENONFINITE
    assert np.array_equal(out["U_new"], np.asarray(case["U_nom"]))
    solver.close()


def test_deterministic_repeat_and_host_api(ora, workloads):
    case = workloads["wall_k4096"][2]
    solver = B.Solver(case["robot"], case["cost"], B.FP32)
    a = device_update(solver, case, 1234, 9, B.FP32)
    b = device_update(solver, case, 1234, 9, B.FP32)
    assert np.array_equal(a["U_new"], b["U_new"]) and np.array_equal(a["costs"], b["costs"])
    st, U_host, S_host = solver.update(case["q0"], case["qd0"], case["target"], case["U_nom"], 1234, 9)
    assert st == B.OK
    assert np.array_equal(U_host, a["U_new"]) and np.array_equal(S_host, a["costs"])
    c = device_update(solver, case, 1234, 10, B.FP32)
    assert not np.array_equal(c["costs"], a["costs"])   # the tick word changes the noise
    solver.close()


def test_plant_step_matches_oracle(ora, workloads):
    torch, dev = torch_dev()
    for case in workloads["wall_k4096"][:3]:
        solver = B.Solver(case["robot"], case["cost"], B.FP32)
        rng = np.random.default_rng(5)
        u = np.array(case["U_nom"][0]) + rng.normal(size=7) * 3
        q = torch.tensor(case["q0"], dtype=torch.float64, device=dev)
        qd = torch.tensor(case["qd0"], dtype=torch.float64, device=dev)
        ut = torch.tensor(u, dtype=torch.float64, device=dev)
        qr, qdr = np.array(case["q0"]), np.array(case["qd0"])
        for _ in range(5):
            solver.plant_step_async(q, qd, ut, 0.01, 10)
            qr, qdr = ora.plant_step(case["robot"], case["cost"], qr, qdr, u, 0.01, 10)
        torch.cuda.synchronize()
        assert np.abs(q.cpu().numpy() - qr).max() < 1e-9
        assert np.abs(qd.cpu().numpy() - qdr).max() < 1e-8
        solver.close()


def test_stage_entry_points_compose_to_the_fused_update(ora, workloads):
    """rollout_async (costs, noise) followed by weights_async gives the fused
    update's U_new; the fused kernel's merged per-wave partials equal the
    one-pass weighting up to rounding."""
    torch, dev = torch_dev()
    case = workloads["wall_k4096"][4]
    solver = B.Solver(case["robot"], case["cost"], B.FP32)
    fused = device_update(solver, case, 55, 2, B.FP32)
    io = fused["io"]
    U_fused = io["U_new"].clone()
    io["U_new"].fill_(float("nan"))
    solver.rollout_async(io)
    solver.weights_async(io)
    torch.cuda.synchronize()
    assert np.abs(io["U_new"].cpu().numpy() - U_fused.cpu().numpy()).max() < 1e-5
    solver.close()


@pytest.mark.parametrize("K", [16384, 20000])
def test_many_block_merge(ora, workloads, K):
    """Hundreds of partials merged by the last block (K/64 waves)."""
    case = workloads["wall_k4096"][5]
    cost = dict(case["cost"], K=K, T=6)
    case = dict(case, cost=cost, U_nom=np.array(case["U_nom"])[:6])
    solver = B.Solver(case["robot"], cost, B.FP32)
    out = device_update(solver, case, 7, 1, B.FP32)
    U_ref, S_ref, _ = oracle_update(ora, case, cost, 7, 1)
    check_costs_fp32(ora, case, out["costs"], S_ref, 7, 1, "K=%d" % K)
    note = check_update(ora, case, out, 1.0, S_ref, U_ref, "K=%d" % K)
    if note:
        print(note)
    solver.close()


def test_maximum_sample_count(ora, workloads):
    """K = 2^20 (the largest K a solver accepts), T = 18, contact cost, FP32:
    200 sampled costs against the oracle's rollouts of those samples, the
    noise of those samples, and U_new against the oracle's Eq. 4 on the
    GPU's own K costs and noise (stage-isolated criterion)."""
    case = workloads["wall_k4096"][6]
    K = 1 << 20
    cost = dict(case["cost"], K=K)
    solver = B.Solver(case["robot"], cost, B.FP32)
    out = device_update(solver, dict(case, cost=cost), case["seed"], 2, B.FP32)
    solver.close()
    assert out["status"] == B.OK
    ks = np.random.default_rng(11).choice(K, 200, replace=False)
    ks[:2] = [0, K - 1]
    S_ref = np.zeros(len(ks))
    for i, k in enumerate(ks):
        S_ref[i], E_k = ora.rollout(case["robot"], cost, case["target"], case["q0"], case["qd0"], case["U_nom"],
                                    case["seed"], 2, int(k))
        assert np.abs(out["noise"][k] - E_k).max() <= 5e-5
    sub = dict(case, cost=cost)
    flagged = check_costs_fp32(ora, sub, out["costs"][ks], S_ref, case["seed"], 2, "K=2^20")
    assert len(flagged) <= 2
    st, U_stage, _ = ora.weights_update(out["costs"], out["noise"], case["U_nom"], cost["lambda"])
    assert st == 0 and np.abs(out["U_new"] - U_stage).max() <= U_ATOL


@pytest.mark.parametrize("precision", [B.FP32, B.FP64])
def test_maximum_horizon(ora, workloads, precision):
    """T = 256 (the largest horizon) at K = 320 (five waves), position task,
    dt = 2 ms (a 0.512 s horizon: at 10 ms random torques drive most
    trajectories past FP32 range): every sample against the oracle; the
    weighting regenerates the noise (the tile does not fit in LDS)."""
    base = workloads["single_k256"][7]
    U = np.asarray(base["U_nom"])
    U = np.concatenate([U] * 15)[:256]
    cost = dict(base["cost"], K=320, T=256, dt=0.002)
    case = dict(base, cost=cost, U_nom=U.tolist())
    solver = B.Solver(case["robot"], cost, precision)
    out = device_update(solver, case, case["seed"], 3, precision)
    solver.close()
    U_ref, S_ref, E_ref = oracle_update(ora, case, cost, case["seed"], 3)
    assert out["status"] == B.OK
    if precision == B.FP64:
        assert cost_rel_err(out["costs"], S_ref).max() <= 1e-9
        assert np.abs(out["noise"] - E_ref).max() <= 1e-12
    else:
        check_costs_fp32(ora, case, out["costs"], S_ref, case["seed"], 3, "T=256")
        assert np.abs(out["noise"] - E_ref).max() <= 5e-5
    note = check_update(ora, case, out, cost["lambda"], S_ref, U_ref, "T=256")
    if note:
        print(note)


@pytest.mark.parametrize("which,i,K,T,extra", [("wall_k4096", 0, 4096, 18, {}), ("wall_k4096", 1, 4097, 3, {}),
                                               ("wall_k4096", 2, 65, 1, {"noise_rho": 0.7}),
                                               ("collision_k4096", 0, 4096, 18, {}),
                                               ("wall_k4096", 3, 640, 40, {}),
                                               ("single_k256", 0, 256, 18, {}),
                                               ("single_k256", 1, 1000, 5, {"noise_rho": 0.5})])
def test_two_wave_update_equals_one_wave(workloads, which, i, K, T, extra):
    """The two-wave update (dynamics on one wave, noise, force estimate and
    cost on the other) computes every sample as the one-wave update does:
    costs, noise and U_new equal to FP32 rounding (the oracle parity of the default
    launch is covered by the other tests)."""
    base = workloads[which][i]
    U = np.asarray(base["U_nom"])
    U = np.concatenate([U] * (T // len(U) + 1))[:T]
    cost = dict(base["cost"], K=K, T=T, **extra)
    case = dict(base, cost=cost, U_nom=U.tolist())
    outs = []
    for w in (1, 2):
        solver = B.Solver(case["robot"], cost, B.FP32)
        solver.set_launch(w)
        outs.append(device_update(solver, case, case["seed"], 12, B.FP32))
        solver.close()
    one, two = outs
    assert one["status"] == two["status"] == B.OK
    assert np.array_equal(one["noise"], two["noise"])
    rel = cost_rel_err(two["costs"], one["costs"])
    print("%s[%d] K=%d T=%d: max rel cost difference %.3g, bitwise equal %s"
          % (which, i, K, T, rel.max(), np.array_equal(one["costs"], two["costs"])))
    assert rel.max() <= 1e-6
    assert np.abs(one["U_new"] - two["U_new"]).max() <= 1e-6
    assert np.array_equal(one["U_shift"][:-1], two["U_shift"][:-1]) or \
        np.abs(one["U_shift"] - two["U_shift"]).max() <= 1e-6


@pytest.mark.parametrize("waves", [1, 2])
def test_fused_update_with_every_cost_non_finite(workloads, waves):
    """Nominal torques of 1e30 N m overflow every sample's cost: the fused
    update (one-wave and two-wave launches) reports MPPI_ENONFINITE and
    passes the nominal sequence through unchanged, its shift included."""
    case = workloads["wall_k4096"][2]
    cost = dict(case["cost"], K=1000)
    U = np.full((cost["T"], 7), 1e30)
    solver = B.Solver(case["robot"], cost, B.FP32)
    solver.set_launch(waves)
    out = device_update(solver, dict(case, cost=cost), case["seed"], 1, B.FP32, U_nom=U)
    solver.close()
    assert out["status"] == B.ENONFINITE
    assert not np.isfinite(out["costs"]).any()
    assert np.array_equal(out["U_new"], U)
    assert np.array_equal(out["U_shift"][:-1], U[1:]) and np.array_equal(out["U_shift"][-1], U[-1])
