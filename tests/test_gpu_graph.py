"""One device update (mppi_update_async) captured into a HIP graph on a
torch capture stream: the eight-lane rollout launch and its merge launch
(launch 8), or the one fused launch with its device-scope counter, which
the last wave resets (launch 2).  Neither records a memory-set node.  Every
replay must reproduce the eager update with the same inputs bit for bit
(U_new, U_shift, costs, status), also with eager updates of other ticks and
synchronisations between the replays."""
import numpy as np
import pytest

from paper_2609_02020_amd import binding as B
from gpu_util import torch_dev

pytestmark = pytest.mark.gpu


def make_io(torch, dev, case, K, T, tick):
    f64 = dict(dtype=torch.float64, device=dev)
    return {
        "q": torch.tensor(case["q0"], **f64),
        "qd": torch.tensor(case["qd0"], **f64),
        "target": torch.tensor(B.target_vector(case["target"]), **f64),
        "U_nominal": torch.tensor(np.asarray(case["U_nom"], dtype=np.float64), **f64).contiguous(),
        "U_new": torch.full((T, 7), float("nan"), **f64),
        "U_shift": torch.full((T, 7), float("nan"), **f64),
        "costs": torch.full((K,), float("nan"), dtype=torch.float32, device=dev),
        "status": torch.full((1,), -1, dtype=torch.int32, device=dev),
        "seed": case["seed"], "tick": tick,
    }


def host(io):
    return {k: io[k].cpu().numpy().copy() for k in ("U_new", "U_shift", "costs", "status")}


@pytest.mark.parametrize("which,launch", [("wall_k4096", 8), ("collision_k4096", 8), ("wall_k4096", 2)])
def test_graph_replays_equal_eager(workloads, which, launch):
    torch, dev = torch_dev()
    case = workloads[which][0]
    K, T = case["cost"]["K"], case["cost"]["T"]
    print("case %s[0], launch %d, K=%d, T=%d" % (which, launch, K, T), flush=True)
    solver = B.Solver(case["robot"], case["cost"], B.FP32)
    solver.set_launch(launch)
    ref_io = make_io(torch, dev, case, K, T, tick=5)
    solver.update_async(ref_io)
    torch.cuda.synchronize()
    ref = host(ref_io)
    assert int(ref["status"][0]) == B.OK

    gio = make_io(torch, dev, case, K, T, tick=5)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        solver.update_async(gio, side)          # warm-up on a side stream, not captured
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        solver.update_async(gio, torch.cuda.current_stream())
    torch.cuda.synchronize()

    other = make_io(torch, dev, case, K, T, tick=9)
    for r in range(3):
        for key in ("U_new", "U_shift", "costs"):
            gio[key].fill_(float("nan"))
        gio["status"].fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        got = host(gio)
        for key in ("U_new", "U_shift", "costs", "status"):
            assert np.array_equal(got[key], ref[key]), (r, key)
        # eager work between the replays
        solver.update_async(other)
        torch.cuda.synchronize()
        assert int(other["status"].cpu()[0]) == B.OK
        assert not np.array_equal(other["U_new"].cpu().numpy(), ref["U_new"])
    graph.reset()
    solver.close()
