"""Closed loop at a torque-interface rate above the solver rate.

The paper's controller sends torques at about 166 Hz to a 1 kHz torque
interface and bridges the gap with a zero-order hold (Sec. IV-A).  This
loop reproduces that structure for any solver period: the FP64 plant is
integrated in plant_ms steps, the solver runs every period_ms on the
current state, the first row of its U_new is held until the next command,
and the warm start of the next update is U_new advanced by the elapsed time
(period / dt horizon steps, mppi_batch_warm_start_async).  A command is
applied at once (delay = 0) or one solver period late (delay = 1: the
latency of a solver that needs its whole period to compute).

Everything here sequences library calls on one stream (binding.Batch:
updates, warm starts, plant steps); torch holds device memory.  Episodes run
side by side as the problems of one batch.
"""
from __future__ import annotations

import numpy as np

from . import binding as B


def run(robot, cost, episodes, K, period_ms, seconds, delay=0, plant_ms=1.0, stream=None):
    """Runs len(episodes) episodes of `seconds` each.  Returns numpy arrays
    q, qd [steps + 1][n][7] (plant state every plant_ms, from the start), u
    [steps][n][7] (torque held over each plant step) and the status words,
    plus the solver-tick count."""
    import torch
    assert torch.cuda.is_available(), "the closed loop needs a GPU"
    dev = torch.device("cuda:0")
    if delay not in (0, 1):
        raise ValueError("delay is 0 or 1 solver periods")
    per = int(round(period_ms / plant_ms))
    if per < 1 or abs(per * plant_ms - period_ms) > 1e-9:
        raise ValueError("the solver period must be a multiple of the plant step")
    n, T, dt = len(episodes), int(cost["T"]), float(cost["dt"])
    batch = B.Batch([(robot, dict(cost, K=int(K)))] * n)
    f64 = dict(dtype=torch.float64, device=dev)
    U0 = np.array([np.asarray(e["U_nom"], dtype=np.float64)[:T] for e in episodes]).reshape(n * T, 7)
    io = {"q": torch.tensor(np.array([e["q0"] for e in episodes]), **f64),
          "qd": torch.tensor(np.array([e["qd0"] for e in episodes]), **f64),
          "target": torch.tensor(np.array([B.target_vector(e["target"]) for e in episodes]), **f64),
          "U_nominal": torch.tensor(U0, **f64), "U_new": torch.empty((n * T, 7), **f64),
          "status": torch.zeros(n, dtype=torch.int32, device=dev),
          "seed": torch.tensor([int(e["seed"]) for e in episodes], dtype=torch.int64, device=dev)}
    held = torch.tensor(U0, **f64)      # first rows: the command being applied
    pending = torch.tensor(U0, **f64)   # delay = 1: the command of the last solve
    plant = dict(io, U_new=held)        # the plant reads the first rows of U_new
    steps = int(round(seconds * 1e3 / plant_ms))
    q = torch.empty((steps + 1, n, 7), **f64)
    qd = torch.empty((steps + 1, n, 7), **f64)
    u = torch.empty((steps, n, 7), **f64)
    shift = period_ms * 1e-3 / dt
    q[0].copy_(io["q"])
    qd[0].copy_(io["qd"])
    ticks = 0
    for s in range(steps):
        if s % per == 0:
            batch.update_async(io, tick=ticks, stream=stream)
            ticks += 1
            if delay:
                held.copy_(pending)
                pending.copy_(io["U_new"])
            else:
                held.copy_(io["U_new"])
            batch.warm_start_async(io["U_new"], io["U_nominal"], shift, stream=stream)
        u[s].copy_(held.view(n, T * 7)[:, :7])
        batch.plant_step_async(plant, plant_ms * 1e-3, 1, stream=stream)
        q[s + 1].copy_(io["q"])
        qd[s + 1].copy_(io["qd"])
    torch.cuda.synchronize()
    out = {"q": q.cpu().numpy(), "qd": qd.cpu().numpy(), "u": u.cpu().numpy(),
           "status": io["status"].cpu().numpy(), "ticks": ticks}
    batch.close()
    return out
