"""The autotuners and their cache: mppi_autotune (single problem, launch
shapes 8, 2, 1) and mppi_batch_autotune (one or eight lanes per sample x
workgroup sizes x resident waves) store their choice in the JSON cache
file set by mppi_set_autotune_cache, keyed by architecture, sizes,
precision and cost terms; a later tuner with the same key takes the stored
shape without timing (times reported as -1), a different key or no cache
times again, and the file stays valid JSON."""
import json

import numpy as np
import pytest

from paper_2609_02020_amd import binding as B
from gpu_util import device_update, torch_dev
from test_gpu_batch import batch_io, small_cases

pytestmark = pytest.mark.gpu


def solver_io(case, torch, dev):
    f64 = dict(dtype=torch.float64, device=dev)
    K, T = case["cost"]["K"], case["cost"]["T"]
    return {"q": torch.tensor(case["q0"], **f64), "qd": torch.tensor(case["qd0"], **f64),
            "target": torch.tensor(B.target_vector(case["target"]), **f64),
            "U_nominal": torch.tensor(case["U_nom"], **f64), "U_new": torch.zeros((T, 7), **f64),
            "costs": torch.zeros(K, dtype=torch.float32, device=dev), "seed": case["seed"], "tick": 3}


def test_solver_autotune_and_cache(ora, workloads, tmp_path):
    torch, dev = torch_dev()
    path = tmp_path / "tune.json"
    B.set_autotune_cache(path)
    try:
        case = workloads["wall_k4096"][0]
        solver = B.Solver(case["robot"], case["cost"], B.FP32)
        best, times = solver.autotune(solver_io(case, torch, dev), budget_ms=30)
        print("single problem K=4096 T=18: launch %d, times (8, 2, 1) %s ms" % (best, np.round(times, 4)))
        assert best in (8, 2, 1) and all(t > 0 for t in times)
        assert times[(8, 2, 1).index(best)] == min(times)
        # eight lanes per sample is the fastest shape at this K by a wide margin
        assert best == 8
        entries = json.load(open(path))
        key = [k for k in entries if k.startswith("solver|")]
        assert len(key) == 1 and entries[key[0]]["waves_per_group"] == best and "|K4096|T18|fp32|" in key[0]
        # the same key again: taken from the cache, no timing
        solver2 = B.Solver(case["robot"], case["cost"], B.FP32)
        solver2.set_launch(1)
        best2, times2 = solver2.autotune(solver_io(case, torch, dev), budget_ms=30)
        assert best2 == best and times2 == [-1.0] * 3
        out = device_update(solver2, case, case["seed"], 5, B.FP32)   # runs on the cached shape
        assert out["status"] == B.OK
        solver.close()
        solver2.close()
        # another K is another key: timed
        small = dict(case, cost=dict(case["cost"], K=512))
        s3 = B.Solver(small["robot"], small["cost"], B.FP32)
        _, times3 = s3.autotune(solver_io(small, torch, dev), budget_ms=15)
        assert all(t > 0 for t in times3)
        s3.close()
        assert len([k for k in json.load(open(path)) if k.startswith("solver|")]) == 2
    finally:
        B.set_autotune_cache(None)


def test_batch_autotune_cache_round_trip(workloads, tmp_path):
    torch, dev = torch_dev()
    path = tmp_path / "tune.json"
    B.set_autotune_cache(path)
    try:
        cases = small_cases(workloads, 6, tmax=16)
        batch = B.Batch([(c["robot"], c["cost"]) for c in cases])
        io = batch_io(batch, cases, torch, dev)
        w, g, times = batch.autotune(io, reps=1)
        assert all(t > 0 for t in times)
        batch.close()
        entries = json.load(open(path))
        key = [k for k in entries if k.startswith("batch|")]
        assert len(key) == 1
        assert (entries[key[0]]["waves_per_group"], entries[key[0]]["groups"]) == (w, g)
        batch2 = B.Batch([(c["robot"], c["cost"]) for c in cases])
        io2 = batch_io(batch2, cases, torch, dev)
        w2, g2, times2 = batch2.autotune(io2, reps=1)
        assert (w2, g2) == (w, g) and times2 == [-1.0] * 16
        batch2.close()
    finally:
        B.set_autotune_cache(None)
    # without the cache the tuner times again
    batch3 = B.Batch([(c["robot"], c["cost"]) for c in cases])
    _, _, times3 = batch3.autotune(batch_io(batch3, cases, torch, dev), reps=1)
    assert all(t > 0 for t in times3)
    batch3.close()
