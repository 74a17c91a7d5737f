"""GPU parity of the warm start for a solver period that differs from dt
(single problem and batch) against the oracle's mean of the held
sequence; s = 1 reproduces an update's U_shift bit for bit."""
import numpy as np
import pytest

from paper_2609_02020_amd import binding as B
from gpu_util import device_update, torch_dev

pytestmark = pytest.mark.gpu


def test_warm_start_matches_oracle(ora, workloads):
    torch, dev = torch_dev()
    case = workloads["wall_k4096"][0]
    solver = B.Solver(case["robot"], dict(case["cost"], K=256), B.FP32)
    U = np.random.default_rng(7).normal(size=(18, 7)) * 4
    Ud = torch.tensor(U, dtype=torch.float64, device=dev)
    out = torch.empty_like(Ud)
    for s in (0.0, 0.1, 0.6, 1.0, 1.5, 2.0, 7.25, 17.0, 17.9, 18.0):
        solver.warm_start_async(Ud, out, s)
        torch.cuda.synchronize()
        ref = ora.warm_start(U, s)
        assert np.abs(out.cpu().numpy() - ref).max() <= 1e-14 * np.abs(U).max(), s
        if float(s).is_integer():
            assert np.array_equal(out.cpu().numpy(), ref), s
    for bad in (-0.5, 18.5, float("nan")):
        with pytest.raises(B.MppiError) as e:
            solver.warm_start_async(Ud, out, bad)
        assert e.value.status == B.EINVAL
    big = torch.zeros((19, 7), dtype=torch.float64, device=dev)
    with pytest.raises(B.MppiError) as e:
        solver.warm_start_async(big[:18], big[1:], 0.5)   # overlapping buffers of full size
    assert e.value.status == B.EINVAL
    with pytest.raises(ValueError):
        solver.warm_start_async(Ud, Ud[1:], 0.5)   # one row short: refused before the library
    solver.close()


def test_one_step_equals_the_update_shift(workloads):
    torch, dev = torch_dev()
    case = workloads["wall_k4096"][1]
    solver = B.Solver(case["robot"], case["cost"], B.FP32)
    out = device_update(solver, case, case["seed"], 4, B.FP32)
    Un = torch.tensor(out["U_new"], dtype=torch.float64, device=dev)
    W = torch.empty_like(Un)
    solver.warm_start_async(Un, W, 1.0)
    torch.cuda.synchronize()
    assert np.array_equal(W.cpu().numpy(), out["U_shift"])
    solver.close()


def test_batch_warm_start_matches_oracle(ora, workloads):
    torch, dev = torch_dev()
    cases = workloads["batch64"][:6]
    batch = B.Batch([(c["robot"], dict(c["cost"], K=256)) for c in cases])
    rng = np.random.default_rng(8)
    U = rng.normal(size=(batch.u_total // 7, 7))
    Ud = torch.tensor(U, dtype=torch.float64, device=dev)
    out = torch.full_like(Ud, float("nan"))
    for s in (0.6, 1.0, 3.3):
        batch.warm_start_async(Ud, out, s)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        for p, c in enumerate(cases):
            u0, T = batch.u_off[p] // 7, c["cost"]["T"]
            ref = ora.warm_start(U[u0:u0 + T], s)
            assert np.abs(got[u0:u0 + T] - ref).max() <= 1e-14 * np.abs(U).max(), (p, s)
    batch.close()
