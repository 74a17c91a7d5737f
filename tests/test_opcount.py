"""The algorithmic flop count the benchmark divides by: the rollout kernel's
per-sample code run on the host with an op-counting scalar."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import bench
from paper_2609_02020_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def oc(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    so = str(tmp_path_factory.mktemp("oc") / "libopcount.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2609_02020_amd", "csrc"),
                    os.path.join(ROOT, "tests", "opcount.cpp"), "-o", so], check=True)
    return C.CDLL(so)


def counts(oc, case, T):
    D = C.POINTER(C.c_double)
    rp = B.robot_params(case["robot"])
    cp = B.cost_params(dict(case["cost"], T=T))
    tgt = B.target_vector(case["target"])
    U = np.ascontiguousarray(np.tile(np.array(case["U_nom"])[0], (T, 1)))
    out = (C.c_longlong * 6)()
    q0 = np.ascontiguousarray(case["q0"], dtype=float)
    qd0 = np.ascontiguousarray(case["qd0"], dtype=float)
    oc.oc_rollout(C.byref(rp), C.byref(cp), tgt.ctypes.data_as(D), q0.ctypes.data_as(D),
                  qd0.ctypes.data_as(D), U.ctypes.data_as(D), T, out)
    return np.array(list(out))


def per_step(oc, case):
    a, b = counts(oc, case, 1), counts(oc, case, 2)
    step = b - a
    return int(step[:4].sum()), int((a - step)[:4].sum())


def test_bench_flop_constants_match_count(oc, workloads):
    step, term = per_step(oc, workloads["wall_k4096"][0])
    assert step == bench.FLOPS_PER_SAMPLE_STEP
    assert term == bench.FLOPS_PER_SAMPLE_TERMINAL
    # the count is a property of the code path, not of the inputs
    for case in workloads["wall_k4096"][1:4]:
        assert per_step(oc, case) == (step, term)


def test_bench_flop_constants_free_space(oc, workloads):
    """The free-space problems of the batched workload (no wall, no force or
    orientation cost) take the shorter path."""
    free = [c for c in workloads["batch64"] if not bench.has_force(c["cost"])]
    assert free
    for case in free[:4]:
        assert per_step(oc, case) == (bench.FLOPS_PER_SAMPLE_STEP_FREE, bench.FLOPS_PER_SAMPLE_TERMINAL_FREE)


def test_mlp_flop_constants():
    """2 flops per weight per row forward; training adds the backward
    products of layers 4..2 and the weight gradients."""
    from oracle import mlp as om
    weights = sum(shape[0] * shape[1] for _, shape, _ in om.layer_slices())
    assert bench.MLP_FWD_FLOPS_PER_ROW == 2 * weights
    assert bench.MLP_TRAIN_FLOPS_PER_ROW == 4 * weights + 2 * (weights - 21 * 256)


def test_bench_flop_constant_explicit_route(oc, workloads):
    """The paper's dynamics route (M by Eq. 8, Cholesky) on the contact
    workload."""
    for case in workloads["wall_k4096"][:3]:
        c = dict(case, cost=dict(case["cost"], dynamics=B.DYN_EXPLICIT_M))
        assert per_step(oc, c) == (bench.FLOPS_PER_SAMPLE_STEP_EXPLICIT, bench.FLOPS_PER_SAMPLE_TERMINAL)
