"""CPU check of the rollout kernels' per-sample math against the oracle.

tests/hostcheck.cpp compiles the kernels' header-only math (dyn.hpp,
rollout.hpp, model_prep.hpp) for the host with g++; these tests compare it,
in FP64 and FP32, with the oracle on the same seeded inputs.  This catches
algebra mistakes on the CPU before any GPU run; the GPU parity tests are in
test_gpu_parity.py.
"""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2609_02020_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hc(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    so = str(tmp_path_factory.mktemp("hc") / "libhostcheck.so")
    subprocess.run(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-pthread",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2609_02020_amd", "csrc"),
                    os.path.join(ROOT, "tests", "hostcheck.cpp"), "-o", so], check=True)
    L = C.CDLL(so)
    D = C.POINTER(C.c_double)
    L.hc_step.argtypes = [C.POINTER(B.RobotParams), C.POINTER(B.CostParams), C.c_int, C.c_int,
                          C.c_int, D, D, D, D, D, D, D, D]
    L.hc_rollout.argtypes = [C.POINTER(B.RobotParams), C.POINTER(B.CostParams), C.c_int, D, D, D,
                             D, C.c_uint64, C.c_uint64, C.c_uint32, D]
    L.hc_rollout.restype = C.c_double
    L.hc_normals.argtypes = [C.c_int, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, D]
    L.hc_seg_dist2.argtypes = [C.c_int, D, D, D, D]
    L.hc_seg_dist2.restype = C.c_double
    L.hc_collision.argtypes = [C.POINTER(B.RobotParams), C.POINTER(B.CostParams), C.c_int, D]
    L.hc_collision.restype = C.c_double
    L.hc_group_step.argtypes = L.hc_step.argtypes
    L.hc_group_rollout.argtypes = L.hc_rollout.argtypes
    L.hc_group_rollout.restype = C.c_double
    L.hc_group_rollout_split.argtypes = L.hc_rollout.argtypes
    L.hc_group_rollout_split.restype = C.c_double
    return L


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(C.POINTER(C.c_double))


def step(hc, case, prec, force, ext, q, qd, tau, v):
    rp = B.robot_params(case["robot"])
    cp = B.cost_params(case["cost"], prec)
    qdd, pee, Rn, F = np.zeros(7), np.zeros(3), np.zeros(9), np.zeros(6)
    args = [np.ascontiguousarray(x, dtype=np.float64) for x in (q, qd, tau, v)]
    hc.hc_step(C.byref(rp), C.byref(cp), prec, force, ext, *[_d(a) for a in args],
               qdd.ctypes.data_as(C.POINTER(C.c_double)), pee.ctypes.data_as(C.POINTER(C.c_double)),
               Rn.ctypes.data_as(C.POINTER(C.c_double)), F.ctypes.data_as(C.POINTER(C.c_double)))
    return qdd, pee, Rn.reshape(3, 3), F


@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-10), (B.FP32, 2e-4)])
def test_aba_step_matches_oracle(hc, ora, workloads, prec, tol):
    rng = np.random.default_rng(11)
    for case in workloads["single_k256"][:6]:
        q = rng.uniform(-2, 2, 7)
        qd = rng.uniform(-2, 2, 7)
        tau = rng.uniform(-20, 20, 7)
        qdd, pee, Rn, _ = step(hc, case, prec, 0, 0, q, qd, tau, tau)
        ref = ora.aba(case["robot"], q, qd, tau)
        scale = np.abs(ref).max() + 1.0
        assert np.abs(qdd - ref).max() < tol * scale
        _, _, pe_ref, _ = ora.fk(case["robot"], q)
        R_ref, _, _, _ = ora.fk(case["robot"], q)
        assert np.abs(pee - pe_ref).max() < tol
        assert np.abs(Rn - R_ref[-1]).max() < tol


@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-9), (B.FP32, 5e-4)])
def test_wall_step_and_force_estimate_match_oracle(hc, ora, workloads, prec, tol):
    rng = np.random.default_rng(12)
    for case in workloads["wall_k4096"][:5]:
        rb, cost = case["robot"], case["cost"]
        q = np.array(case["q0"]) + rng.uniform(-0.3, 0.3, 7)
        qd = rng.uniform(-1, 1, 7)
        v = rng.uniform(-10, 10, 7)
        # push the EE into the wall so the contact force is active
        _, _, pe, _ = ora.fk(rb, q)
        cost = dict(cost, wall_d0=float(np.dot(cost["wall_n"], pe)) + 0.01)
        case2 = dict(case, cost=cost)
        qdd, _, _, F = step(hc, case2, prec, 1, 2, q, qd, v, v)
        J = ora.ee_jacobian(rb, q)
        fw = np.concatenate([ora.wall_force(cost, pe, J[:3] @ qd), np.zeros(3)])
        assert np.linalg.norm(fw) > 1.0
        ref = ora.aba(rb, q, qd, v, fw)
        assert np.abs(qdd - ref).max() < tol * (np.abs(ref).max() + 1)
        g = ora.bias_jacobian(rb, q, np.zeros(7))
        Fref = ora.force_estimate(rb, q, v - g)
        assert np.abs(F - Fref).max() < tol * (np.abs(Fref).max() + 1) * 10


@pytest.mark.parametrize("prec", [B.FP64, B.FP32])
def test_normals_match_oracle(hc, ora, prec):
    for (seed, tick, k, t) in [(3000, 0, 0, 0), (2**40 + 17, 123456789, 4095, 17), (7, 5, 77, 3)]:
        z = np.zeros(8)
        hc.hc_normals(prec, seed, tick, k, t, z.ctypes.data_as(C.POINTER(C.c_double)))
        ref = ora.normals(seed, tick, k, t)
        tol = 1e-13 if prec == B.FP64 else 2e-5
        assert np.abs(z - ref).max() < tol * (1 + np.abs(ref).max())


@pytest.mark.parametrize("which", ["single_k256", "wall_k4096"])
@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-9), (B.FP32, 1e-4)])
def test_rollout_cost_matches_oracle(hc, ora, workloads, which, prec, tol):
    for case in workloads[which][:3]:
        rp = B.robot_params(case["robot"])
        cp = B.cost_params(case["cost"], prec)
        tgt = B.target_vector(case["target"])
        U = np.ascontiguousarray(case["U_nom"], dtype=np.float64)
        for k in (0, 5, 1234):
            noise = np.zeros((case["cost"]["T"], 7))
            S = hc.hc_rollout(C.byref(rp), C.byref(cp), prec, _d(tgt), _d(case["q0"]),
                              _d(case["qd0"]), _d(U), case["seed"], 3, k,
                              noise.ctypes.data_as(C.POINTER(C.c_double)))
            S_ref, n_ref = ora.rollout(case["robot"], case["cost"], case["target"], case["q0"],
                                       case["qd0"], U, case["seed"], 3, k)
            assert abs(S - S_ref) <= tol * abs(S_ref), (S, S_ref)
            assert np.abs(noise - n_ref).max() < (1e-12 if prec == B.FP64 else 1e-4)


def test_force_estimate_through_the_handoff(hc, workloads):
    """The two-wave update hands the force-estimate inputs over through a
    flat buffer: every slot of the layout is written (no NaN left), and the
    estimate formed from the buffer equals the inline one (FP64)."""
    D = C.POINTER(C.c_double)
    hc.hc_step_handoff.argtypes = [C.POINTER(B.RobotParams), C.POINTER(B.CostParams), D, D, D, D, D, D, D]
    rng = np.random.default_rng(5)
    for case in workloads["wall_k4096"][:4]:
        rp = B.robot_params(case["robot"])
        cp = B.cost_params(case["cost"], B.FP64)
        for _ in range(3):
            q = np.asarray(case["q0"]) + rng.uniform(-0.3, 0.3, 7)
            qd = rng.uniform(-1, 1, 7)
            tau = rng.normal(size=7) * 5
            F, Fs, dq = np.zeros(6), np.zeros(6), np.zeros(1)
            hc.hc_step_handoff(C.byref(rp), C.byref(cp), _d(q), _d(qd), _d(tau), _d(tau),
                               F.ctypes.data_as(D), Fs.ctypes.data_as(D), dq.ctypes.data_as(D))
            assert np.isfinite(Fs).all() and dq[0] == 0.0
            assert np.array_equal(F, Fs)


@pytest.mark.parametrize("rho", [0.5, 0.95])
@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-9), (B.FP32, 1e-4)])
def test_correlated_noise_rollout_matches_oracle(hc, ora, workloads, rho, prec, tol):
    """AR(1) perturbation in time (noise_step) against the oracle's recursion."""
    for which in ("single_k256", "wall_k4096"):
        case = workloads[which][0]
        cost = dict(case["cost"], noise_rho=rho)
        rp = B.robot_params(case["robot"])
        cp = B.cost_params(cost, prec)
        tgt = B.target_vector(case["target"])
        U = np.ascontiguousarray(case["U_nom"], dtype=np.float64)
        for k in (0, 77):
            noise = np.zeros((cost["T"], 7))
            S = hc.hc_rollout(C.byref(rp), C.byref(cp), prec, _d(tgt), _d(case["q0"]), _d(case["qd0"]), _d(U),
                              case["seed"], 3, k, noise.ctypes.data_as(C.POINTER(C.c_double)))
            S_ref, n_ref = ora.rollout(case["robot"], cost, case["target"], case["q0"], case["qd0"], U,
                                       case["seed"], 3, k)
            assert abs(S - S_ref) <= tol * abs(S_ref), (S, S_ref)
            assert np.abs(noise - n_ref).max() < (1e-12 if prec == B.FP64 else 1e-4)
            # the recursion is in effect: later steps differ from the independent draws
            _, n_iid = ora.rollout(case["robot"], case["cost"], case["target"], case["q0"], case["qd0"], U,
                                   case["seed"], 3, k)
            assert np.array_equal(n_ref[0], n_iid[0]) and np.abs(n_ref[1:] - n_iid[1:]).max() > 1e-3


def _dp(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(C.POINTER(C.c_double))


@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-12), (B.FP32, 2e-5)])
def test_segment_distance_matches_oracle(hc, ora, prec, tol):
    """The kernels' clamped closest-point construction against the oracle's
    minimisation over the unit square, including parallel, crossing and
    point-like segments."""
    rng = np.random.default_rng(2)
    cases = [rng.normal(size=(4, 3)) for _ in range(400)]
    a = np.array([0.0, 0, 0])
    cases += [np.array([a, [1, 0, 0], [0.5, 0.3, 0], [2, 0.3, 0]]),      # parallel overlap
              np.array([a, [1, 0, 0], [2, 0.3, 0], [3, 0.3, 0]]),        # parallel apart
              np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0]]),   # crossing
              np.array([[0.5, 2, 0], [0.5, 2, 0], a, [1, 0, 0]]),        # a is a point
              np.array([a, [1, 0, 0], [3, 1, 0], [3, 1, 0]]),            # b is a point
              np.array([[1, 1, 1]] * 4)]                                   # both points, same
    for s in cases:
        ref = ora.segment_distance(*s)
        got = np.sqrt(hc.hc_seg_dist2(prec, *(_dp(x) for x in s)))
        assert abs(got - ref) <= tol * max(1.0, ref), (s, got, ref)


def collision_cost_dict(case, rng):
    """Self pairs of non-adjacent links and link-obstacle pairs against two
    vertical obstacles near the start configuration."""
    pe = np.asarray(case["target"]["p_des"])
    obstacles = [[pe[0] + 0.15, pe[1], pe[2] - 0.3, pe[0] + 0.15, pe[1], pe[2] + 0.3],
                 [pe[0], pe[1] - 0.25, 0.0, pe[0], pe[1] - 0.25, 1.0]]
    pairs = [[i, j] for i in range(7) for j in range(i + 2, 7)][:12]
    pairs += [[i, 7 + o] for o in range(2) for i in (3, 4, 5, 6)]
    d_th = [0.08] * 12 + [0.2] * 8
    return dict(case["cost"], w_collision=3e4, obstacles=obstacles, pairs=pairs, d_th=d_th)


@pytest.mark.parametrize("prec", [B.FP64, B.FP32])
def test_collision_cost_matches_oracle(hc, ora, workloads, prec):
    rng = np.random.default_rng(3)
    compared = 0
    for case in workloads["wall_k4096"][:5]:
        cost = collision_cost_dict(case, rng)
        rp = B.robot_params(case["robot"])
        cp = B.cost_params(cost, prec)
        for _ in range(40):
            q = np.asarray(case["q0"]) + rng.uniform(-0.8, 0.8, 7)
            ref, margin = ora.collision_cost(case["robot"], cost, q)
            if margin < (1e-9 if prec == B.FP64 else 1e-4):
                continue   # an indicator that rounding may flip
            assert hc.hc_collision(C.byref(rp), C.byref(cp), prec, _dp(q)) == ref
            compared += 1
    assert compared > 150


@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-10), (B.FP32, 2e-4)])
def test_explicit_m_step_matches_oracle(hc, ora, workloads, prec, tol):
    """The paper's route (M by Eq. 8, Cholesky) against the oracle's forward
    dynamics, with and without the wall, and its force estimate."""
    rng = np.random.default_rng(21)
    for case in workloads["wall_k4096"][:5]:
        rb = case["robot"]
        q = np.array(case["q0"]) + rng.uniform(-0.5, 0.5, 7)
        qd = rng.uniform(-2, 2, 7)
        v = rng.uniform(-15, 15, 7)
        _, _, pe, _ = ora.fk(rb, q)
        cost = dict(case["cost"], dynamics=B.DYN_EXPLICIT_M,
                    wall_d0=float(np.dot(case["cost"]["wall_n"], pe)) + 0.01)
        case2 = dict(case, cost=cost)
        # free motion
        qdd, pee, Rn, _ = step(hc, case2, prec, 0, 0, q, qd, v, v)
        ref = ora.forward_dynamics(rb, q, qd, v)
        assert np.abs(qdd - ref).max() < tol * (np.abs(ref).max() + 1)
        assert np.abs(pee - pe).max() < tol
        # wall contact + force estimate
        qdd, _, _, F = step(hc, case2, prec, 1, 2, q, qd, v, v)
        J = ora.ee_jacobian(rb, q)
        fw = np.concatenate([ora.wall_force(cost, pe, J[:3] @ qd), np.zeros(3)])
        assert np.linalg.norm(fw) > 1.0
        ref = ora.forward_dynamics(rb, q, qd, v, fw)
        assert np.abs(qdd - ref).max() < tol * (np.abs(ref).max() + 1)
        g = ora.bias_jacobian(rb, q, np.zeros(7))
        Fref = ora.force_estimate(rb, q, v - g)
        assert np.abs(F - Fref).max() < tol * (np.abs(Fref).max() + 1) * 10


def test_explicit_m_rollout_matches_oracle(hc, ora, workloads):
    """Whole FP64 rollouts of the contact workload on the explicit route."""
    D = C.POINTER(C.c_double)
    for case in workloads["wall_k4096"][:3]:
        cost = dict(case["cost"], dynamics=B.DYN_EXPLICIT_M)
        rp, cp = B.robot_params(case["robot"]), B.cost_params(cost, B.FP64)
        tgt = B.target_vector(case["target"])
        U = np.ascontiguousarray(case["U_nom"], dtype=np.float64)
        noise = np.zeros(18 * 7)
        for k in (0, 5, 77):
            S = hc.hc_rollout(C.byref(rp), C.byref(cp), B.FP64, tgt.ctypes.data_as(D),
                              _dp(case["q0"]), _dp(case["qd0"]), U.ctypes.data_as(D), case["seed"], 2, k,
                              noise.ctypes.data_as(D))
            ref, _ = ora.rollout(case["robot"], case["cost"], case["target"], case["q0"], case["qd0"],
                                 case["U_nom"], case["seed"], 2, k)
            assert abs(S - ref) <= 1e-9 * abs(ref)


# ---------------------------------------------------------------------------
# the eight-lanes-per-sample rollout (group.hpp), run on eight host threads
# ---------------------------------------------------------------------------
def group_step(hc, case, prec, force, ext, q, qd, tau, v):
    rp = B.robot_params(case["robot"])
    cp = B.cost_params(case["cost"], prec)
    qdd, pee, Re, F = np.zeros(7), np.zeros(3), np.zeros(9), np.zeros(6)
    args = [np.ascontiguousarray(x, dtype=np.float64) for x in (q, qd, tau, v)]
    hc.hc_group_step(C.byref(rp), C.byref(cp), prec, force, ext, *[_d(a) for a in args],
                     qdd.ctypes.data_as(C.POINTER(C.c_double)), pee.ctypes.data_as(C.POINTER(C.c_double)),
                     Re.ctypes.data_as(C.POINTER(C.c_double)), F.ctypes.data_as(C.POINTER(C.c_double)))
    return qdd, pee, Re.reshape(3, 3), F


@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-10), (B.FP32, 2e-4)])
def test_group_step_matches_oracle(hc, ora, workloads, prec, tol):
    """One step on the lane group (scans, composite-rigid-body M, LDL^T)
    against the oracle's forward dynamics and kinematics (free motion), and
    with the wall in contact against its dynamics and the force estimate of
    Eq. 13 (taken about the EE point)."""
    rng = np.random.default_rng(31)
    for case in workloads["wall_k4096"][:5]:
        rb = case["robot"]
        q = np.array(case["q0"]) + rng.uniform(-0.5, 0.5, 7)
        qd = rng.uniform(-2, 2, 7)
        v = rng.uniform(-15, 15, 7)
        R_ref, _, pe, _ = ora.fk(rb, q)
        cost = dict(case["cost"], wall_d0=float(np.dot(case["cost"]["wall_n"], pe)) + 0.01)
        case2 = dict(case, cost=cost)
        qdd, pee, Re, _ = group_step(hc, case2, prec, 0, 0, q, qd, v, v)
        ref = ora.forward_dynamics(rb, q, qd, v)
        assert np.abs(qdd - ref).max() < tol * (np.abs(ref).max() + 1)
        assert np.abs(pee - pe).max() < tol
        Ree = np.asarray(rb["R_ee"]).reshape(3, 3)
        assert np.abs(Re - R_ref[-1] @ Ree).max() < tol
        qdd, _, _, F = group_step(hc, case2, prec, 1, 2, q, qd, v, v)
        J = ora.ee_jacobian(rb, q)
        fw = np.concatenate([ora.wall_force(cost, pe, J[:3] @ qd), np.zeros(3)])
        assert np.linalg.norm(fw) > 1.0
        ref = ora.forward_dynamics(rb, q, qd, v, fw)
        assert np.abs(qdd - ref).max() < tol * (np.abs(ref).max() + 1)
        g = ora.bias_jacobian(rb, q, np.zeros(7))
        Fref = ora.force_estimate(rb, q, v - g)
        assert np.abs(F - Fref).max() < tol * (np.abs(Fref).max() + 1)


@pytest.mark.parametrize("split", [False, True])
@pytest.mark.parametrize("which", ["single_k256", "wall_k4096"])
@pytest.mark.parametrize("prec,tol", [(B.FP64, 1e-9), (B.FP32, 1e-4)])
def test_group_rollout_cost_matches_oracle(hc, ora, workloads, which, prec, tol, split):
    """Whole rollouts on the lane group: every lane ends with the same total
    (the host function returns NaN otherwise), equal to the oracle's S_k;
    the noise of every joint equals the oracle's.  split: each step as its
    dynamics part and then its cost part, the factor of M handed over in
    the group area (the eight-lane batch kernel's path)."""
    fn = hc.hc_group_rollout_split if split else hc.hc_group_rollout
    for case in workloads[which][:3]:
        rp = B.robot_params(case["robot"])
        cp = B.cost_params(case["cost"], prec)
        tgt = B.target_vector(case["target"])
        U = np.ascontiguousarray(case["U_nom"], dtype=np.float64)
        for k in (0, 5, 1234):
            noise = np.zeros((case["cost"]["T"], 7))
            S = fn(C.byref(rp), C.byref(cp), prec, _d(tgt), _d(case["q0"]), _d(case["qd0"]), _d(U),
                   case["seed"], 3, k, noise.ctypes.data_as(C.POINTER(C.c_double)))
            S_ref, n_ref = ora.rollout(case["robot"], case["cost"], case["target"], case["q0"],
                                       case["qd0"], U, case["seed"], 3, k)
            assert abs(S - S_ref) <= tol * abs(S_ref), (S, S_ref)
            assert np.abs(noise - n_ref).max() < (1e-12 if prec == B.FP64 else 1e-4)


def test_group_rollout_variants_match_oracle(hc, ora, workloads):
    """FP64 group rollouts with correlated noise, the literal tau_F and the
    constant external wrench."""
    D = C.POINTER(C.c_double)
    base = workloads["wall_k4096"][2]
    for extra in ({"noise_rho": 0.7}, {"force_mode": 1},
                  {"ext_mode": 1, "F_ext": [3.0, -2.0, 5.0, 0.2, -0.1, 0.3]}):
        cost = dict(base["cost"], **extra)
        rp, cp = B.robot_params(base["robot"]), B.cost_params(cost, B.FP64)
        tgt = B.target_vector(base["target"])
        U = np.ascontiguousarray(base["U_nom"], dtype=np.float64)
        noise = np.zeros((cost["T"], 7))
        for k in (0, 9):
            S = hc.hc_group_rollout(C.byref(rp), C.byref(cp), B.FP64, tgt.ctypes.data_as(D), _d(base["q0"]),
                                    _d(base["qd0"]), U.ctypes.data_as(D), base["seed"], 1, k,
                                    noise.ctypes.data_as(D))
            S_ref, _ = ora.rollout(base["robot"], cost, base["target"], base["q0"], base["qd0"], U,
                                   base["seed"], 1, k)
            assert abs(S - S_ref) <= 1e-9 * abs(S_ref), (extra, S, S_ref)


@pytest.mark.parametrize("split", [False, True])
def test_group_rollout_with_collision_term_matches_oracle(hc, ora, workloads, split):
    """FP64 group rollouts of the collision workload (Eqs. 14-15, pairs dealt
    over the lanes) against the oracle's rollouts."""
    D = C.POINTER(C.c_double)
    fn = hc.hc_group_rollout_split if split else hc.hc_group_rollout
    for case in workloads["collision_k4096"][:2]:
        rp, cp = B.robot_params(case["robot"]), B.cost_params(case["cost"], B.FP64)
        assert cp.n_pairs > 8   # more pairs than lanes
        tgt = B.target_vector(case["target"])
        U = np.ascontiguousarray(case["U_nom"], dtype=np.float64)
        noise = np.zeros((case["cost"]["T"], 7))
        for k in (0, 3, 100):
            S = fn(C.byref(rp), C.byref(cp), B.FP64, tgt.ctypes.data_as(D), _d(case["q0"]), _d(case["qd0"]),
                   U.ctypes.data_as(D), case["seed"], 2, k, noise.ctypes.data_as(D))
            S_ref, _ = ora.rollout(case["robot"], case["cost"], case["target"], case["q0"], case["qd0"], U,
                                   case["seed"], 2, k)
            assert abs(S - S_ref) <= 1e-9 * abs(S_ref), (k, S, S_ref)
