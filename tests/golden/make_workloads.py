"""Write tests/golden/workloads.json: the seeded synthetic workloads.

Calls only the seeded generators (paper_2609_02020_amd.inputs) and the CPU
oracle (oracle/).  Run from the repository root:

    python tests/golden/make_workloads.py

Recipe (all seeds fixed):
  * arm i: draw_arm(1000 + i + 100000 a), state: draw_state(2000 + i +
    100000 a) for the first attempt a that passes the acceptance test:
    |g_j(q)| <= 0.6 tau_max,j at q0 and at the goal configuration and
    sigma_min(J(q0)) >= 0.05 (no singular start).
  * target pose = FK(q_goal); wall (contact cases): normal among +-x/+-y,
    plane 0.02-0.05 m beyond the initial EE point along -n, desired force
    10 N into the wall (F_des = -10 n).
  * initial nominal U_nom[t] = g(q0) for every step (gravity compensation).
  * Philox key = 3000 + case index (single updates) / episode.
  * collision_k4096: wall_k4096[0..3] with the collision term (see
    with_collision()).
  * learned_wall.json: the learned-proposal task (see learned_wall()).
  * free_space.json: the free-space hybrid task (see free_space());
    `python tests/golden/make_workloads.py free_space` writes only it.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np
from scipy.spatial.transform import Rotation

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as ora  # noqa: E402
from paper_2609_02020_amd import inputs  # noqa: E402


def accepted_case(index: int, arm_base: int = 1000, state_base: int = 2000):
    for attempt in range(50):
        arm = inputs.draw_arm(arm_base + index + 100000 * attempt)
        q0, qd0, qg = inputs.draw_state(state_base + index + 100000 * attempt)
        lim = np.array([L["tau_max"] for L in arm["links"]])
        g0 = ora.bias_jacobian(arm, q0, np.zeros(7))
        g1 = ora.bias_jacobian(arm, qg, np.zeros(7))
        smin = np.linalg.svd(ora.ee_jacobian(arm, q0), compute_uv=False).min()
        if (np.abs(g0) <= 0.6 * lim).all() and (np.abs(g1) <= 0.6 * lim).all() and smin >= 0.05:
            return arm, q0, qd0, qg
    raise RuntimeError("no acceptable arm for case %d" % index)


def target_of(arm, q_goal, F_des=None):
    _, _, pe, Re = ora.fk(arm, q_goal)
    x, y, z, w = Rotation.from_matrix(Re).as_quat()
    return {"p_des": pe.tolist(), "quat_des": [float(w), float(x), float(y), float(z)],
            "F_des": list(F_des) if F_des is not None else [0.0] * 6}


def make_case(index, kind, K, T, dt, lam, seed, arm_base=1000, state_base=2000,
              wall_seed=None):
    arm, q0, qd0, qg = accepted_case(index, arm_base, state_base)
    g0 = ora.bias_jacobian(arm, q0, np.zeros(7))
    if kind == "position":
        cost = inputs.position_cost(K, T, dt, lam)
        target = target_of(arm, qg)
    else:
        normal, axis, standoff = inputs.draw_wall(wall_seed if wall_seed is not None else 7000 + index)
        _, _, pe0, _ = ora.fk(arm, q0)
        d0 = float(np.dot(normal, pe0) - standoff)
        cost = inputs.wall_cost(K, T, normal, axis, d0, dt, lam)
        F_des = [-10.0 * n for n in normal] + [0.0, 0.0, 0.0]
        target = target_of(arm, qg, F_des)
    U_nom = np.tile(g0, (T, 1))
    return {"kind": kind, "robot": arm, "cost": cost, "target": target,
            "q0": list(map(float, q0)), "qd0": list(map(float, qd0)),
            "q_goal": list(map(float, qg)), "U_nom": U_nom.tolist(),
            "seed": int(seed), "tick": 0}


def gravity_stable(arm, q, tol=0.5):
    """The arm hangs at q: every eigenvalue of M^-1 dg/dq (g the gravity
    torque, central differences) is >= -tol, so no configuration mode is
    pushed away from q by gravity."""
    M = ora.crba(arm, q)
    h = 1e-6
    G = np.array([(ora.bias_jacobian(arm, q + e, np.zeros(7)) - ora.bias_jacobian(arm, q - e, np.zeros(7))) / (2 * h)
                  for e in np.eye(7) * h]).T
    return np.linalg.eigvals(np.linalg.solve(M, G)).real.min() >= -tol


def learned_wall(n_train=1000, n_eval=50):
    """The learned-proposal task: the arm and wall normal of wall_k4096[0];
    the base posture is the first of draw_postures(1, 20000) that passes the
    gravity and Jacobian acceptance tests and is gravity-stable (the arm
    hangs); the wall plane lies 0.03 m beyond the base EE point along -n.
    Every episode starts at base + draw_perturbation (+-0.2 rad start,
    +-0.3 rad goal) with qd0 = 0, U_nom = g(q0), the target pose FK(goal)
    and 10 N into the wall, accepted when the gravity torques at start and
    goal are within 0.6 tau_max, sigma_min(J(q0)) >= 0.05 and the start EE
    point lies 0-0.08 m in front of the wall.  Cost: the wall cost of the
    contact workload with the velocity-limit penalty on (w_qd = 1e4) and
    lambda = 10."""
    base = make_case(100, "wall", 4096, 18, 0.01, 1.0, 3000)
    arm = base["robot"]
    n = np.array(base["cost"]["wall_n"])
    lim = np.array([L["tau_max"] for L in arm["links"]])

    def gravity_ok(q):
        return (np.abs(ora.bias_jacobian(arm, q, np.zeros(7))) <= 0.6 * lim).all()

    def smin(q):
        return np.linalg.svd(ora.ee_jacobian(arm, q), compute_uv=False).min()

    qb = next(q for q in inputs.draw_postures(1, 20000)
              if gravity_ok(q) and gravity_stable(arm, q) and smin(q) >= 0.05)
    _, _, peb, _ = ora.fk(arm, qb)
    d0 = float(n @ peb - 0.03)
    axis = int(np.argmax(np.abs(n)))
    cost = inputs.wall_cost(4096, 18, n.tolist(), axis, d0, 0.01, 10.0)
    cost["w_qd"] = 1e4
    F_des = [-10.0 * v for v in n] + [0.0, 0.0, 0.0]
    eps = []
    for e in range(n_train + n_eval):
        for attempt in range(200):
            dq0, dqg = inputs.draw_perturbation(6000 + e + 100000 * attempt)
            q0, qg = qb + dq0, qb + dqg
            _, _, pe, _ = ora.fk(arm, q0)
            if gravity_ok(q0) and gravity_ok(qg) and smin(q0) >= 0.05 and 0.0 <= n @ pe - d0 <= 0.08:
                break
        else:
            raise RuntimeError("no acceptable episode %d" % e)
        eps.append({"q0": q0.tolist(), "qd0": [0.0] * 7, "target": target_of(arm, qg, F_des),
                    "g0": ora.bias_jacobian(arm, q0, np.zeros(7)).tolist(), "seed": 5000 + e})
    return {"robot": arm, "cost": cost, "q_base": qb.tolist(), "train": eps[:n_train], "eval": eps[n_train:]}


def free_space(n=8, learned_path=None):
    """The free-space hybrid task of Sec. IV-B: the arm and base posture of
    the learned-proposal task (read from learned_wall.json); episode e
    starts at base + the start offset of draw_perturbation(8000 + e +
    100000 a) (+-0.2 rad) for the first attempt a whose gravity torques are
    within 0.6 tau_max and sigma_min(J(q0)) >= 0.05, at rest, with
    U_nom = g(q0); the target is a step reference from the start pose: the
    EE point raised 0.03 m along z (the position-controlled axes are y and
    z), the initial orientation, and 10 N along +x (F_des = (10, 0, 0, 0,
    0, 0)); the posture term's rest posture is the start configuration
    (q_rest = q0, stored with the episode).  Cost: inputs.free_space_cost
    (K = 4096, T = 18, dt = 0.01 s, lambda = 1)."""
    lw = inputs.load_learned(learned_path) if learned_path else inputs.load_learned()
    arm, qb = lw["robot"], np.array(lw["q_base"])
    lim = np.array([L["tau_max"] for L in arm["links"]])
    eps = []
    for e in range(n):
        for attempt in range(200):
            dq0, _ = inputs.draw_perturbation(8000 + e + 100000 * attempt)
            q0 = qb + dq0
            g0 = ora.bias_jacobian(arm, q0, np.zeros(7))
            smin = np.linalg.svd(ora.ee_jacobian(arm, q0), compute_uv=False).min()
            if (np.abs(g0) <= 0.6 * lim).all() and smin >= 0.05:
                break
        else:
            raise RuntimeError("no acceptable free-space episode %d" % e)
        tg = target_of(arm, q0, [10.0, 0.0, 0.0, 0.0, 0.0, 0.0])
        tg["p_des"][2] += 0.03
        eps.append({"q0": q0.tolist(), "qd0": [0.0] * 7, "target": tg, "g0": g0.tolist(), "q_rest": q0.tolist(),
                    "seed": 9000 + e})
    return {"robot": arm, "cost": inputs.free_space_cost(4096, 18, 0.01, 1.0), "episodes": eps}


def write_free_space():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "free_space.json")
    with open(path, "w") as f:
        json.dump(free_space(), f, indent=None, separators=(",", ":"))
    print("wrote", path, os.path.getsize(path), "bytes")


def with_collision(case):
    """The contact case plus the collision term of Eqs. 14-15: two vertical
    obstacle segments beside the target point (0.15 m along +x, 0.25 m
    along -y), the 12 first pairs of non-adjacent links (threshold 0.08 m)
    and links 3-6 against both obstacles (threshold 0.2 m, the paper's
    safety distance); w_collision = 3e4 (Table I)."""
    pe = np.asarray(case["target"]["p_des"])
    obstacles = [[pe[0] + 0.15, pe[1], pe[2] - 0.3, pe[0] + 0.15, pe[1], pe[2] + 0.3],
                 [pe[0], pe[1] - 0.25, 0.0, pe[0], pe[1] - 0.25, 1.0]]
    pairs = [[i, j] for i in range(7) for j in range(i + 2, 7)][:12]
    pairs += [[i, 7 + o] for o in range(2) for i in (3, 4, 5, 6)]
    cost = dict(case["cost"], w_collision=3e4, obstacles=obstacles, pairs=pairs,
                d_th=[0.08] * 12 + [0.2] * 8)
    return dict(case, cost=cost)


def main():
    out = {"recipe": __doc__.strip().splitlines()[0]}
    # single update, position cost, K=256, T=18, dt=0.01, lambda=1 (FP64 case)
    out["single_k256"] = [make_case(i, "position", 256, 18, 0.01, 1.0, 3000 + i) for i in range(20)]
    # closed loop with a wall, K=4096, T=18, dt=0.01, lambda=1 (FP32 case)
    out["wall_k4096"] = [make_case(100 + e, "wall", 4096, 18, 0.01, 1.0, 3000 + e) for e in range(10)]
    # precision study: K=16384, T=36, dt=0.005, lambda in {0.01, 0.1, 1}
    out["precision_k16384"] = [make_case(100, "wall", 16384, 36, 0.005, lam, 3100 + i)
                               for i, lam in enumerate((0.01, 0.1, 1.0))]
    # batched: 64 problems, K ~ U{512..8192}, T ~ U{10..50}, half position / half wall
    Ks, Ts = inputs.draw_horizon(4000, 64)
    out["batch64"] = [make_case(200 + i, "position" if i % 2 == 0 else "wall", Ks[i], Ts[i],
                                0.01, 1.0, 3200 + i) for i in range(64)]
    # contact task with the collision term, K=4096, T=18
    out["collision_k4096"] = [with_collision(c) for c in out["wall_k4096"][:4]]
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "workloads.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=None, separators=(",", ":"))
    print("wrote", path, os.path.getsize(path), "bytes")
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "learned_wall.json")
    with open(path, "w") as f:
        json.dump(learned_wall(), f, indent=None, separators=(",", ":"))
    print("wrote", path, os.path.getsize(path), "bytes")
    write_free_space()


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "free_space":
        write_free_space()
    else:
        main()
