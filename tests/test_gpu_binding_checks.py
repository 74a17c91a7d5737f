"""The binding refuses device tensors that do not fit what the kernels
read and write (the C ABI takes raw pointers and cannot check them): wrong
element type, too few elements, a non-contiguous view, a host tensor.
Each refusal happens before any launch, and the solver still works after."""
import numpy as np
import pytest

from paper_2609_02020_amd import binding as B
from gpu_util import device_update, torch_dev

pytestmark = pytest.mark.gpu


def test_solver_io_checks(workloads):
    torch, dev = torch_dev()
    case = workloads["single_k256"][0]
    solver = B.Solver(case["robot"], case["cost"], B.FP32)
    K, T = solver.K, solver.T
    f64 = dict(dtype=torch.float64, device=dev)

    def io(**over):
        d = {"q": torch.tensor(case["q0"], **f64), "qd": torch.tensor(case["qd0"], **f64),
             "target": torch.tensor(B.target_vector(case["target"]), **f64),
             "U_nominal": torch.tensor(case["U_nom"], **f64), "U_new": torch.zeros((T, 7), **f64),
             "costs": torch.zeros(K, dtype=torch.float32, device=dev), "seed": 1, "tick": 0}
        d.update(over)
        return d

    bad = [
        {"costs": torch.zeros(K, **f64)},                                   # FP64 costs, FP32 solver
        {"costs": torch.zeros(K - 1, dtype=torch.float32, device=dev)},     # one element short
        {"U_new": torch.zeros((7, T), **f64).t()},                          # non-contiguous view
        {"q": torch.tensor(case["q0"], dtype=torch.float64)},               # host memory
        {"noise": torch.zeros(T * 7 * K - 1, dtype=torch.float32, device=dev)},
        {"status": torch.zeros(1, dtype=torch.int64, device=dev)},
    ]
    for over in bad:
        with pytest.raises(ValueError):
            solver.update_async(io(**over))
    # still a working solver
    out = device_update(solver, case, case["seed"], 0, B.FP32)
    assert out["status"] == B.OK and np.isfinite(out["costs"]).all()
    solver.close()


def test_network_and_batch_io_checks(workloads):
    torch, dev = torch_dev()
    case = workloads["single_k256"][0]
    net = B.Mlp(case["robot"], 64)
    x = torch.zeros((8, B.MLP_INPUTS), dtype=torch.float32, device=dev)
    with pytest.raises(ValueError):
        net.forward_async(x, torch.zeros((7, B.MLP_OUTPUTS), dtype=torch.float32, device=dev))
    with pytest.raises(ValueError):
        net.forward_async(x.double(), torch.zeros((8, B.MLP_OUTPUTS), dtype=torch.float32, device=dev))
    q = torch.zeros((4, 7), dtype=torch.float64, device=dev)
    with pytest.raises(ValueError):   # U too short for 4 proposals of 126 values
        net.propose_async(q, q, torch.zeros((4, 13), dtype=torch.float64, device=dev),
                          torch.zeros(3 * 126, dtype=torch.float64, device=dev))
    net.close()
    cases = [dict(c, cost=dict(c["cost"], K=300)) for c in workloads["batch64"][:2]]
    batch = B.Batch([(c["robot"], c["cost"]) for c in cases])
    with pytest.raises(ValueError):   # seeds must be 64-bit integers
        batch.update_async({"q": torch.zeros((2, 7), dtype=torch.float64, device=dev),
                            "seed": torch.zeros(2, dtype=torch.int32, device=dev)}, tick=0)
    batch.close()
