"""Seeded synthetic input generators shared by the tests and the benchmark.

This module only draws random numbers and lays them out as plain dicts; it
holds none of the method's arithmetic (no kinematics, dynamics, costs or
weighting).  Quantities that need the robot model (target poses from a goal
configuration, wall placement, the initial gravity-compensating nominal and
the arm acceptance test) are computed once by ``tests/golden/make_workloads.py``
with the CPU oracle and stored in ``tests/golden/workloads.json``; ``load``
reads that file.

Arm family (a stand-in for the 7-DoF arm of the paper, whose parameters are
not published): a serial chain of 7 revolute joints about local z; joint 1
vertical, every later joint frame turned by Rx(+-pi/2); link lengths
U[0.1, 0.4] m with a lateral offset U[-0.1, 0.1] m; masses U[0.5, 4] kg;
CoM near the link axis at 0.3-0.7 of its length; inertia of a solid box
(extents U[0.04, 0.1] x U[0.04, 0.1] x length) turned by a random rotation
(positive definite and satisfying the triangle inequality by construction);
armature U[0.02, 0.1] kg m^2; limits q in [-2.8, 2.8] rad, |qd| <= 2.5
rad/s, |tau| <= 87 N m (joints 1-4) / 12 N m (joints 5-7).
"""
from __future__ import annotations

import json
import os

import numpy as np
from scipy.spatial.transform import Rotation

NJ = 7
TAU_MAX = [87.0, 87.0, 87.0, 87.0, 12.0, 12.0, 12.0]
WORKLOADS_JSON = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                              "tests", "golden", "workloads.json")
LEARNED_JSON = os.path.join(os.path.dirname(WORKLOADS_JSON), "learned_wall.json")

_RX_PLUS = [[1.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]]
_RX_MINUS = [[1.0, 0.0, 0.0], [0.0, 0.0, 1.0], [0.0, -1.0, 0.0]]
_EYE = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]]


def draw_arm(seed: int, n: int = NJ) -> dict:
    """Random arm parameters (see module docstring)."""
    rng = np.random.default_rng(seed)
    lengths = rng.uniform(0.1, 0.4, size=n)
    links = []
    for i in range(n):
        if i == 0:
            R_parent = _EYE
            r_parent = [0.0, 0.0, float(rng.uniform(0.1, 0.3))]
        else:
            R_parent = _RX_PLUS if rng.integers(0, 2) else _RX_MINUS
            r_parent = [float(rng.uniform(-0.1, 0.1)), 0.0, float(lengths[i - 1])]
        L = float(lengths[i])
        m = float(rng.uniform(0.5, 4.0))
        com = [float(rng.uniform(-0.02, 0.02)), float(rng.uniform(-0.02, 0.02)),
               float(rng.uniform(0.3, 0.7) * L)]
        bx, by = rng.uniform(0.04, 0.1, size=2)
        principal = np.diag([m / 12.0 * (by * by + L * L),
                             m / 12.0 * (bx * bx + L * L),
                             m / 12.0 * (bx * bx + by * by)])
        Rc = Rotation.random(random_state=rng).as_matrix()
        I = Rc @ principal @ Rc.T
        links.append({
            "R_parent": [list(map(float, r)) for r in R_parent],
            "r_parent": r_parent,
            "mass": m,
            "com": com,
            "inertia": [float(I[0, 0]), float(I[1, 1]), float(I[2, 2]),
                        float(I[0, 1]), float(I[0, 2]), float(I[1, 2])],
            "armature": float(rng.uniform(0.02, 0.1)),
            "q_min": -2.8, "q_max": 2.8, "qd_max": 2.5,
            "tau_max": TAU_MAX[i] if n == NJ else 87.0,
        })
    return {"n": n, "links": links, "R_ee": _EYE, "r_ee": [0.0, 0.0, 0.1],
            "gravity": [0.0, 0.0, -9.81]}


def draw_state(seed: int, n: int = NJ):
    """q0 ~ U[-1, 1]^n, qd0 = 0, goal configuration q0 + U[-0.5, 0.5]^n."""
    rng = np.random.default_rng(seed)
    q0 = rng.uniform(-1.0, 1.0, size=n)
    q_goal = q0 + rng.uniform(-0.5, 0.5, size=n)
    return q0.tolist(), [0.0] * n, q_goal.tolist()


def draw_wall(seed: int):
    """Wall normal among +-x, +-y and its standoff U[0.02, 0.05] m."""
    rng = np.random.default_rng(seed)
    axis = int(rng.integers(0, 2))
    sign = 1.0 if rng.integers(0, 2) else -1.0
    normal = [0.0, 0.0, 0.0]
    normal[axis] = sign
    return normal, axis, float(rng.uniform(0.02, 0.05))


def draw_horizon(seed: int, count: int):
    """Batched problems: K ~ U{512..8192}, T ~ U{10..50}."""
    rng = np.random.default_rng(seed)
    K = rng.integers(512, 8193, size=count)
    T = rng.integers(10, 51, size=count)
    return K.tolist(), T.tolist()


def position_cost(K: int, T: int, dt: float = 0.01, lam: float = 1.0) -> dict:
    """Plain position task: W_pos = 1e3 I, joint-limit (1e4) and
    torque-limit (10) penalties, terminal weight 1, sigma = 2 N m."""
    return {
        "K": K, "T": T, "dt": dt, "lambda": lam, "sigma": [2.0] * NJ,
        "W_pos": [1e3, 1e3, 1e3], "W_ori": [0.0] * 3,
        "W_force": [0.0] * 6, "W_reg": [0.0] * 6,
        "w_q": 1e4, "w_qd": 0.0, "w_tau": 10.0, "w_post": 0.0,
        "q_rest": [0.0] * NJ, "w_terminal": 1.0, "force_mode": 0,
        "ext_mode": 0, "F_ext": [0.0] * 6, "wall_n": [0.0, 0.0, 0.0],
        "wall_d0": 0.0, "wall_k": 0.0, "wall_c": 0.0,
    }


def wall_cost(K: int, T: int, normal, axis: int, d0: float, dt: float = 0.01,
              lam: float = 1.0) -> dict:
    """Contact task against a planar wall: W_pos = 1e3 on the two axes
    tangent to the wall, W_ori = 1e2, W_force = 0.1 on the normal force
    axis, W_reg = W_force / 30 on all six, spring 2000 N/m, damper 20 N s/m."""
    c = position_cost(K, T, dt, lam)
    W_pos = [1e3, 1e3, 1e3]
    W_pos[axis] = 0.0
    W_force = [0.0] * 6
    W_force[axis] = 0.1
    c.update({"W_pos": W_pos, "W_ori": [1e2] * 3, "W_force": W_force,
              "W_reg": [0.1 / 30.0] * 6, "ext_mode": 2, "wall_n": list(normal),
              "wall_d0": float(d0), "wall_k": 2000.0, "wall_c": 20.0})
    return c


def free_space_cost(K: int, T: int, dt: float = 0.01, lam: float = 1.0) -> dict:
    """Hybrid motion/force task in free space: Table I's free-space weights
    (W_pos diag(0, 5e6, 5e6), W_ori 5e5 I, W_force diag(30, 0, ...), W_reg I)
    scaled by 1e3 / 5e6 to the position weight of the other workloads
    (W_pos = 1e3 on y and z), so W_ori = 100, W_force = 0.006 on the x
    force, W_reg = 2e-4 on all six; joint-limit (1e4), velocity-limit (1e4)
    and torque-limit (10) penalties; the posture term of C_joint on
    (w_post = 10; its rest posture q_rest is set per episode to the start
    configuration); no contact model in the controller."""
    c = position_cost(K, T, dt, lam)
    s = 1e3 / 5e6
    c.update({"W_pos": [0.0, 5e6 * s, 5e6 * s], "W_ori": [5e5 * s] * 3,
              "W_force": [30.0 * s, 0.0, 0.0, 0.0, 0.0, 0.0], "W_reg": [1.0 * s] * 6,
              "w_qd": 1e4, "w_post": 10.0})
    return c


def draw_perturbation(seed: int, n: int = NJ, start_width: float = 0.2, goal_width: float = 0.3):
    """Offsets of a start and a goal configuration, uniform in +-start_width
    and +-goal_width rad per joint."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(-start_width, start_width, size=n).tolist(),
            rng.uniform(-goal_width, goal_width, size=n).tolist())


def draw_postures(seed: int, count: int, n: int = NJ, half_width: float = 2.5) -> np.ndarray:
    """count candidate configurations, uniform in +-half_width rad per joint."""
    rng = np.random.default_rng(seed)
    return np.array([rng.uniform(-half_width, half_width, size=n) for _ in range(count)])


def load(path: str = WORKLOADS_JSON) -> dict:
    """Stored workloads (written by tests/golden/make_workloads.py)."""
    with open(path) as f:
        return json.load(f)


MLP_DIMS = (21, 256, 256, 256, 126)


def draw_mlp_params(seed: int) -> np.ndarray:
    """Initial parameters of the proposal network, flat FP64 in the layout
    W_1, b_1, ..., W_4, b_4 (W_l row-major [out][in]): every entry of layer l
    uniform in +-1/sqrt(fan_in)."""
    rng = np.random.default_rng(seed)
    parts = []
    for n_in, n_out in zip(MLP_DIMS[:-1], MLP_DIMS[1:]):
        s = 1.0 / np.sqrt(n_in)
        parts.append(rng.uniform(-s, s, size=n_out * n_in))
        parts.append(rng.uniform(-s, s, size=n_out))
    return np.concatenate(parts)


def draw_mlp_batch(seed: int, rows: int, scale: float = 1.0):
    """A synthetic regression batch for the network kernels: inputs
    X [rows][21] uniform in +-scale, targets Y [rows][126] uniform in +-0.5."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(-scale, scale, size=(rows, MLP_DIMS[0])),
            rng.uniform(-0.5, 0.5, size=(rows, MLP_DIMS[-1])))


FREE_SPACE_JSON = os.path.join(os.path.dirname(WORKLOADS_JSON), "free_space.json")


def load_free_space(path: str = FREE_SPACE_JSON) -> dict:
    """Episodes of the free-space hybrid task (written by
    tests/golden/make_workloads.py): {"robot", "cost", "episodes": [...]},
    each episode {"q0", "qd0", "target", "U_nom", "seed"}."""
    with open(path) as f:
        d = json.load(f)
    T = d["cost"]["T"]
    for e in d["episodes"]:
        e["U_nom"] = [list(e["g0"])] * T
    return d


def load_learned(path: str = LEARNED_JSON) -> dict:
    """Episodes of the learned-proposal task (one arm, one wall, written by
    tests/golden/make_workloads.py): {"robot", "cost", "train": [...],
    "eval": [...]}, each episode {"q0", "qd0", "target", "U_nom", "seed"}."""
    with open(path) as f:
        d = json.load(f)
    T = d["cost"]["T"]
    for part in ("train", "eval"):
        for e in d[part]:
            e["U_nom"] = [list(e["g0"])] * T
    return d
