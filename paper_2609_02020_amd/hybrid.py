"""Hybrid motion/force control in free space with motion blocking and
pushes (Sec. IV-B, Table I free-space column) on the simulated arm.

The controller is one MPPI solver with the free-space cost: pose on the
position-controlled axes y and z and the orientation, a 10 N force target
along x through the torque-based force estimate of Eq. 13, and no contact
model.  The plant is the FP64 zero-order-hold plant of a second handle of
the same arm, whose external-wrench model stands in for what the
experiment did to the robot:

* motion blocking along the force-controlled axis: a stiff planar wall
  (the contact workload's spring-damper, 2000 N/m and 20 N s/m) through
  the EE point at the moment the block starts, normal against the force
  target (the plane is placed from the EE pose the library computes for the
  current state);
* pushes: a constant world force at the EE point, added to the plant's
  dynamics and unknown to the controller (mppi_plant_step_wrench_async).

Everything here sequences library calls on one stream: updates, plant
steps, EE poses; torch holds device memory.  A tick is one update at the
solver's dt followed by dt of plant time in 1 ms substeps; the warm start is
the shifted U_new.
"""
from __future__ import annotations

import numpy as np

from . import binding as B

# Phases of an episode, in seconds of plant time (the experiment's order:
# free motion under the force target, motion blocking along x, a converged
# free interval, then pushes along +z, +y and -y).  The simulated arm has no
# friction or joint limits to stop a 10 N force target in free space, so
# after the converged interval the blocking wall returns and the pushes act
# with x blocked; the window between blocks is where the experiment's
# errors are reported.
SCHEDULE = {
    "ticks": 400,
    "blocks": [(0.3, 1.0), (1.5, 4.0)],
    "window": (1.0, 1.5),
    "pushes": [(1.7, 2.0, (0.0, 0.0, 1.0)), (2.4, 2.7, (0.0, 1.0, 0.0)), (3.1, 3.4, (0.0, -1.0, 0.0))],
    "push_N": 15.0,
    "block_normal": (-1.0, 0.0, 0.0),
    "wall_k": 2000.0,
    "wall_c": 20.0,
}


def _phase(t, spans):
    for i, span in enumerate(spans):
        if span[0] <= t < span[1]:
            return i
    return -1


def run_episode(robot, cost, episode, schedule=SCHEDULE, K=None, stream=None):
    """One episode of the free-space hybrid task (the episode's q_rest, when
    given, replaces the cost's rest posture).  Returns numpy arrays:
    q, qd [ticks + 1][7] (plant state at every tick), u [ticks][7] (the
    torque held over each tick: the first row of U_new), pose [ticks + 1][7]
    (EE position and quaternion from the library), blocked [ticks] (index of
    the active block or -1), push [ticks] (index of the active push or -1),
    walls [n_blocks][4] (normal and offset d0 of each block's plane) and the
    last status word."""
    import torch
    assert torch.cuda.is_available(), "the free-space scenario needs a GPU"
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    c = dict(cost)
    if "q_rest" in episode:   # the posture term's rest posture of this episode
        c["q_rest"] = list(episode["q_rest"])
    if K is not None:
        c["K"] = int(K)
    T, dt = int(c["T"]), float(c["dt"])
    sub = max(1, int(round(dt / 1e-3)))
    ctrl = B.Solver(robot, c)
    pcost = dict(c, K=1, T=1, ext_mode=B.EXT_NONE)
    plant = B.Solver(robot, pcost)
    io = {"q": torch.tensor(episode["q0"], **f64), "qd": torch.tensor(episode["qd0"], **f64),
          "target": torch.tensor(B.target_vector(episode["target"]), **f64),
          "U_nominal": torch.tensor(np.asarray(episode["U_nom"], dtype=np.float64)[:T], **f64).contiguous(),
          "U_new": torch.empty((T, 7), **f64), "U_shift": torch.empty((T, 7), **f64),
          "status": torch.zeros(1, dtype=torch.int32, device=dev), "seed": int(episode["seed"]), "tick": 0}
    n = int(schedule["ticks"])
    qh = torch.empty((n + 1, 7), **f64)
    qdh = torch.empty((n + 1, 7), **f64)
    uh = torch.empty((n, 7), **f64)
    pose1 = torch.empty(7, **f64)
    wrenches = [torch.tensor([schedule["push_N"] * a for a in p[2]] + [0.0, 0.0, 0.0], **f64)
                for p in schedule["pushes"]]
    nrm = np.asarray(schedule["block_normal"], dtype=np.float64)
    walls = np.zeros((len(schedule["blocks"]), 4))
    blocked = np.full(n, -1, dtype=np.int32)
    pushed = np.full(n, -1, dtype=np.int32)
    qh[0].copy_(io["q"])
    qdh[0].copy_(io["qd"])
    active = -1
    for t in range(n):
        time = t * dt
        b = _phase(time, schedule["blocks"])
        if b != active:
            if b >= 0:
                # the blocking plane through the current EE point
                plant.ee_pose_async(io["q"], pose1, stream=stream)
                p = pose1.cpu().numpy()[:3]
                walls[b, :3], walls[b, 3] = nrm, float(nrm @ p)
                plant.set_cost(dict(pcost, ext_mode=B.EXT_WALL, wall_n=nrm.tolist(), wall_d0=float(walls[b, 3]),
                                    wall_k=schedule["wall_k"], wall_c=schedule["wall_c"]))
            else:
                plant.set_cost(pcost)
            active = b
        blocked[t] = b
        pi = _phase(time, schedule["pushes"])
        pushed[t] = pi
        io["tick"] = t
        ctrl.update_async(io, stream=stream)
        uh[t].copy_(io["U_new"][0])
        plant.plant_step_async(io["q"], io["qd"], uh[t], dt, sub, stream=stream,
                               wrench=wrenches[pi] if pi >= 0 else None)
        qh[t + 1].copy_(io["q"])
        qdh[t + 1].copy_(io["qd"])
        io["U_nominal"], io["U_shift"] = io["U_shift"], io["U_nominal"]
    pose = torch.empty((n + 1, 7), **f64)
    plant.ee_pose_async(qh, pose, stream=stream)
    torch.cuda.synchronize()
    out = {"q": qh.cpu().numpy(), "qd": qdh.cpu().numpy(), "u": uh.cpu().numpy(), "pose": pose.cpu().numpy(),
           "blocked": blocked, "push": pushed, "walls": walls, "status": int(io["status"].cpu()[0]), "dt": dt}
    ctrl.close()
    plant.close()
    return out
