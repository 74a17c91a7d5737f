"""ctypes front end of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check and the CPU-baseline leg of ``bench.py``
import this module.  The product library never does.  The oracle shares no
code with the HIP path; the only thing both sides take is the plain-dict
workload description produced by the seeded input generators
(``robot``/``cost``/``target`` dicts, see ``paper_2609_02020_amd.inputs``).

Every function here is argument marshalling around ``oracle.c``; the
arithmetic, and the passage of the paper each part follows, is there.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
MAXJ = 7
MAXOBS, MAXPAIRS = 4, 32

OK, EINVAL, ENONFINITE, ESINGULAR = 0, 1, 2, 3
EXT_NONE, EXT_CONST, EXT_WALL = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (-O2, OpenMP)."""
    src = os.path.join(HERE, "oracle.c")
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
               src, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Link(C.Structure):
    _fields_ = [("R_parent", C.c_double * 9), ("r_parent", C.c_double * 3),
                ("mass", C.c_double), ("com", C.c_double * 3),
                ("inertia", C.c_double * 6), ("armature", C.c_double),
                ("q_min", C.c_double), ("q_max", C.c_double),
                ("qd_max", C.c_double), ("tau_max", C.c_double)]


class Robot(C.Structure):
    _fields_ = [("n", C.c_int), ("link", Link * MAXJ),
                ("R_ee", C.c_double * 9), ("r_ee", C.c_double * 3),
                ("gravity", C.c_double * 3)]


class Cost(C.Structure):
    _fields_ = [("K", C.c_int), ("T", C.c_int), ("dt", C.c_double),
                ("lam", C.c_double), ("sigma", C.c_double * MAXJ),
                ("W_pos", C.c_double * 3), ("W_ori", C.c_double * 3),
                ("W_force", C.c_double * 6), ("W_reg", C.c_double * 6),
                ("w_q", C.c_double), ("w_qd", C.c_double),
                ("w_tau", C.c_double), ("w_post", C.c_double),
                ("q_rest", C.c_double * MAXJ), ("w_terminal", C.c_double),
                ("force_mode", C.c_int), ("ext_mode", C.c_int),
                ("F_ext", C.c_double * 6), ("wall_n", C.c_double * 3),
                ("wall_d0", C.c_double), ("wall_k", C.c_double),
                ("wall_c", C.c_double), ("w_collision", C.c_double),
                ("n_obstacles", C.c_int), ("obstacles", (C.c_double * 6) * MAXOBS),
                ("n_pairs", C.c_int), ("pairs", (C.c_int * 2) * MAXPAIRS),
                ("d_th", C.c_double * MAXPAIRS),
                ("noise_rho", C.c_double), ("iterations", C.c_int)]


class Target(C.Structure):
    _fields_ = [("p_des", C.c_double * 3), ("quat_des", C.c_double * 4),
                ("F_des", C.c_double * 6)]


_lib = None
_lock = threading.Lock()
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                build()
            L = C.CDLL(LIB_PATH)
            P = C.POINTER
            L.ora_fk.argtypes = [P(Robot), _D, _D, _D, _D, _D]
            L.ora_ee_jacobian.argtypes = [P(Robot), _D, _D]
            L.ora_mass_jacobian_sum.argtypes = [P(Robot), _D, _D]
            L.ora_bias_jacobian.argtypes = [P(Robot), _D, _D, _D]
            L.ora_crba.argtypes = [P(Robot), _D, _D]
            L.ora_rnea.argtypes = [P(Robot), _D, _D, _D, _D, _D]
            L.ora_aba.argtypes = [P(Robot), _D, _D, _D, _D, _D]
            L.ora_forward_dynamics.argtypes = [P(Robot), _D, _D, _D, _D, _D]
            L.ora_forward_dynamics.restype = C.c_int
            L.ora_cholesky_solve.argtypes = [C.c_int, _D, _D]
            L.ora_cholesky_solve.restype = C.c_int
            L.ora_energy.argtypes = [P(Robot), _D, _D]
            L.ora_energy.restype = C.c_double
            L.ora_quat_to_R.argtypes = [_D, _D]
            L.ora_so3_log.argtypes = [_D, _D]
            L.ora_force_estimate.argtypes = [P(Robot), _D, _D, _D]
            L.ora_force_estimate.restype = C.c_int
            L.ora_wall_force.argtypes = [P(Cost), _D, _D, _D]
            L.ora_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
            L.ora_normals.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, _D]
            L.ora_running_cost.argtypes = [P(Robot), P(Cost), P(Target), _D, _D, _D, _D]
            L.ora_running_cost.restype = C.c_double
            L.ora_terminal_cost.argtypes = [P(Robot), P(Cost), P(Target), _D, _D]
            L.ora_terminal_cost.restype = C.c_double
            L.ora_rollout.argtypes = [P(Robot), P(Cost), P(Target), _D, _D, _D,
                                      C.c_uint64, C.c_uint64, C.c_uint32, _D]
            L.ora_rollout.restype = C.c_double
            L.ora_weights_update.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double,
                                             _D, _D, _D, _D, _D]
            L.ora_weights_update.restype = C.c_int
            L.ora_update.argtypes = [P(Robot), P(Cost), P(Target), _D, _D, _D,
                                     C.c_uint64, C.c_uint64, _D, _D, _D, C.c_int]
            L.ora_update.restype = C.c_int
            L.ora_plant_step.argtypes = [P(Robot), P(Cost), _D, _D, _D, C.c_double, C.c_int]
            L.ora_warm_start.argtypes = [C.c_int, C.c_int, _D, C.c_double, _D]
            L.ora_max_threads.restype = C.c_int
            L.ora_segment_distance.argtypes = [_D, _D, _D, _D]
            L.ora_segment_distance.restype = C.c_double
            L.ora_link_segments.argtypes = [P(Robot), _D, _D]
            L.ora_collision_cost.argtypes = [P(Robot), P(Cost), _D, P(C.c_double)]
            L.ora_collision_cost.restype = C.c_double
            L.ora_rollout_margin.argtypes = [P(Robot), P(Cost), P(Target), _D, _D, _D,
                                             C.c_uint64, C.c_uint64, C.c_uint32, _D, P(C.c_double)]
            L.ora_rollout_margin.restype = C.c_double
            _lib = L
    return _lib


# ---------------------------------------------------------------------------
# dict -> struct marshalling
# ---------------------------------------------------------------------------
def _fill(arr, values):
    vals = np.asarray(values, dtype=np.float64).ravel()
    for i, v in enumerate(vals):
        arr[i] = float(v)


def robot_struct(robot: dict) -> Robot:
    rb = Robot()
    rb.n = int(robot["n"])
    for i, L in enumerate(robot["links"]):
        dst = rb.link[i]
        _fill(dst.R_parent, L["R_parent"])
        _fill(dst.r_parent, L["r_parent"])
        dst.mass = float(L["mass"])
        _fill(dst.com, L["com"])
        _fill(dst.inertia, L["inertia"])
        dst.armature = float(L["armature"])
        dst.q_min = float(L["q_min"])
        dst.q_max = float(L["q_max"])
        dst.qd_max = float(L["qd_max"])
        dst.tau_max = float(L["tau_max"])
    _fill(rb.R_ee, robot["R_ee"])
    _fill(rb.r_ee, robot["r_ee"])
    _fill(rb.gravity, robot.get("gravity", [0.0, 0.0, -9.81]))
    return rb


def cost_struct(cost: dict) -> Cost:
    c = Cost()
    c.K = int(cost["K"])
    c.T = int(cost["T"])
    c.dt = float(cost["dt"])
    c.lam = float(cost["lambda"])
    _fill(c.sigma, cost["sigma"])
    for key in ("W_pos", "W_ori", "W_force", "W_reg", "q_rest", "F_ext", "wall_n"):
        _fill(getattr(c, key), cost.get(key, [0.0] * len(getattr(c, key))))
    for key in ("w_q", "w_qd", "w_tau", "w_post", "wall_d0", "wall_k", "wall_c"):
        setattr(c, key, float(cost.get(key, 0.0)))
    c.w_terminal = float(cost.get("w_terminal", 1.0))
    c.force_mode = int(cost.get("force_mode", 0))
    c.ext_mode = int(cost.get("ext_mode", EXT_NONE))
    c.w_collision = float(cost.get("w_collision", 0.0))
    obs = cost.get("obstacles", [])
    pairs = cost.get("pairs", [])
    assert len(obs) <= MAXOBS and len(pairs) <= MAXPAIRS
    c.n_obstacles = len(obs)
    for o, seg in enumerate(obs):
        _fill(c.obstacles[o], seg)
    c.n_pairs = len(pairs)
    for i, (a, b) in enumerate(pairs):
        c.pairs[i][0], c.pairs[i][1] = int(a), int(b)
        c.d_th[i] = float(cost["d_th"][i])
    c.noise_rho = float(cost.get("noise_rho", 0.0))
    c.iterations = int(cost.get("iterations", 1))
    return c


def target_struct(target: dict) -> Target:
    t = Target()
    _fill(t.p_des, target["p_des"])
    _fill(t.quat_des, target.get("quat_des", [1.0, 0.0, 0.0, 0.0]))
    _fill(t.F_des, target.get("F_des", [0.0] * 6))
    return t


def _p(a):
    return a.ctypes.data_as(_D)


def _vec(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if n is not None:
        assert a.size == n, (a.size, n)
    return a


# ---------------------------------------------------------------------------
# numpy-facing wrappers
# ---------------------------------------------------------------------------
def fk(robot, q):
    rb = robot_struct(robot)
    n = rb.n
    q = _vec(q, n)
    R = np.zeros((n, 3, 3)); p = np.zeros((n, 3)); pe = np.zeros(3); Re = np.zeros((3, 3))
    lib().ora_fk(C.byref(rb), _p(q), _p(R), _p(p), _p(pe), _p(Re))
    return R, p, pe, Re


def ee_jacobian(robot, q):
    rb = robot_struct(robot)
    J = np.zeros((6, rb.n))
    lib().ora_ee_jacobian(C.byref(rb), _p(_vec(q, rb.n)), _p(J))
    return J


def mass_jacobian_sum(robot, q):
    rb = robot_struct(robot)
    M = np.zeros((rb.n, rb.n))
    lib().ora_mass_jacobian_sum(C.byref(rb), _p(_vec(q, rb.n)), _p(M))
    return M


def bias_jacobian(robot, q, qd):
    rb = robot_struct(robot)
    h = np.zeros(rb.n)
    lib().ora_bias_jacobian(C.byref(rb), _p(_vec(q, rb.n)), _p(_vec(qd, rb.n)), _p(h))
    return h


def crba(robot, q):
    rb = robot_struct(robot)
    M = np.zeros((rb.n, rb.n))
    lib().ora_crba(C.byref(rb), _p(_vec(q, rb.n)), _p(M))
    return M


def rnea(robot, q, qd, qdd, f_ee=None):
    rb = robot_struct(robot)
    tau = np.zeros(rb.n)
    fe = _vec(f_ee, 6) if f_ee is not None else None
    lib().ora_rnea(C.byref(rb), _p(_vec(q, rb.n)), _p(_vec(qd, rb.n)),
                   _p(_vec(qdd, rb.n)), _p(fe) if fe is not None else None, _p(tau))
    return tau


def aba(robot, q, qd, tau, f_ee=None):
    rb = robot_struct(robot)
    qdd = np.zeros(rb.n)
    fe = _vec(f_ee, 6) if f_ee is not None else None
    lib().ora_aba(C.byref(rb), _p(_vec(q, rb.n)), _p(_vec(qd, rb.n)),
                  _p(_vec(tau, rb.n)), _p(fe) if fe is not None else None, _p(qdd))
    return qdd


def forward_dynamics(robot, q, qd, tau, f_ee=None):
    rb = robot_struct(robot)
    qdd = np.zeros(rb.n)
    fe = _vec(f_ee, 6) if f_ee is not None else None
    st = lib().ora_forward_dynamics(C.byref(rb), _p(_vec(q, rb.n)), _p(_vec(qd, rb.n)),
                                    _p(_vec(tau, rb.n)), _p(fe) if fe is not None else None,
                                    _p(qdd))
    if st:
        raise np.linalg.LinAlgError("mass matrix not positive definite")
    return qdd


def cholesky_solve(A, b):
    A = _vec(A); x = _vec(b).copy()
    st = lib().ora_cholesky_solve(int(x.size), _p(A), _p(x))
    if st:
        raise np.linalg.LinAlgError("not SPD")
    return x


def energy(robot, q, qd):
    rb = robot_struct(robot)
    return lib().ora_energy(C.byref(rb), _p(_vec(q, rb.n)), _p(_vec(qd, rb.n)))


def quat_to_R(quat):
    R = np.zeros((3, 3))
    lib().ora_quat_to_R(_p(_vec(quat, 4)), _p(R))
    return R


def so3_log(R):
    rho = np.zeros(3)
    lib().ora_so3_log(_p(_vec(R, 9)), _p(rho))
    return rho


def force_estimate(robot, q, tau_F):
    rb = robot_struct(robot)
    F = np.zeros(6)
    st = lib().ora_force_estimate(C.byref(rb), _p(_vec(q, rb.n)), _p(_vec(tau_F, rb.n)), _p(F))
    if st:
        raise np.linalg.LinAlgError("singular operational-space inertia")
    return F


def wall_force(cost, p_ee, v_ee):
    c = cost_struct(cost)
    F = np.zeros(3)
    lib().ora_wall_force(C.byref(c), _p(_vec(p_ee, 3)), _p(_vec(v_ee, 3)), _p(F))
    return F


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    out = (C.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, out)
    return [int(x) for x in out]


def normals(seed, tick, k, t):
    z = np.zeros(8)
    lib().ora_normals(C.c_uint64(seed), C.c_uint64(tick), C.c_uint32(k), C.c_uint32(t), _p(z))
    return z


def running_cost(robot, cost, target, q, qd, v):
    rb, c, tg = robot_struct(robot), cost_struct(cost), target_struct(target)
    parts = np.zeros(7)
    total = lib().ora_running_cost(C.byref(rb), C.byref(c), C.byref(tg),
                                   _p(_vec(q, rb.n)), _p(_vec(qd, rb.n)),
                                   _p(_vec(v, rb.n)), _p(parts))
    return total, dict(zip(("pos", "ori", "force", "joint", "torque", "collision", "total"), parts))


def segment_distance(a0, a1, b0, b1):
    return float(lib().ora_segment_distance(*(_p(_vec(x, 3)) for x in (a0, a1, b0, b1))))


def link_segments(robot, q):
    rb = robot_struct(robot)
    seg = np.zeros((rb.n, 6))
    lib().ora_link_segments(C.byref(rb), _p(_vec(q, rb.n)), _p(seg))
    return seg


def collision_cost(robot, cost, q):
    """(C_collision at q, min_i |d_i - d_th,i|)."""
    rb, c = robot_struct(robot), cost_struct(cost)
    m = C.c_double()
    v = lib().ora_collision_cost(C.byref(rb), C.byref(c), _p(_vec(q, rb.n)), C.byref(m))
    return float(v), m.value


def rollout_margin(robot, cost, target, q0, qd0, U_nom, seed, tick, k):
    """(S_k, smallest |d_i - d_th,i| over the horizon's pre-step states)."""
    rb, c, tg = robot_struct(robot), cost_struct(cost), target_struct(target)
    U = _vec(U_nom, c.T * rb.n)
    m = C.c_double()
    S = lib().ora_rollout_margin(C.byref(rb), C.byref(c), C.byref(tg), _p(_vec(q0, rb.n)),
                                 _p(_vec(qd0, rb.n)), _p(U), C.c_uint64(seed), C.c_uint64(tick),
                                 C.c_uint32(k), None, C.byref(m))
    return S, m.value


def terminal_cost(robot, cost, target, q, qd):
    rb, c, tg = robot_struct(robot), cost_struct(cost), target_struct(target)
    return lib().ora_terminal_cost(C.byref(rb), C.byref(c), C.byref(tg),
                                   _p(_vec(q, rb.n)), _p(_vec(qd, rb.n)))


def rollout(robot, cost, target, q0, qd0, U_nom, seed, tick, k):
    rb, c, tg = robot_struct(robot), cost_struct(cost), target_struct(target)
    U = _vec(U_nom, c.T * rb.n)
    noise = np.zeros((c.T, rb.n))
    S = lib().ora_rollout(C.byref(rb), C.byref(c), C.byref(tg), _p(_vec(q0, rb.n)),
                          _p(_vec(qd0, rb.n)), _p(U), C.c_uint64(seed),
                          C.c_uint64(tick), C.c_uint32(k), _p(noise))
    return S, noise


def weights_update(S, noise, U_nom, lam):
    S = _vec(S)
    noise = _vec(noise)
    K = S.size
    T, n = np.asarray(U_nom).shape
    assert noise.size == K * T * n
    U_nom = _vec(U_nom)
    U_new = np.zeros((T, n))
    w = np.zeros(K)
    st = lib().ora_weights_update(K, T, n, float(lam), _p(S), _p(noise), _p(U_nom),
                                  _p(U_new), _p(w))
    return st, U_new, w


def update(robot, cost, target, q0, qd0, U_nom, seed, tick, nthreads=0,
           want_noise=True):
    """One MPPI update (cost["iterations"] chained iterations, one if absent).
    Returns (status, U_new[T,n], costs[K], noise[K,T,n]) of the last iteration."""
    rb, c, tg = robot_struct(robot), cost_struct(cost), target_struct(target)
    K, T, n = c.K, c.T, rb.n
    U = _vec(U_nom, T * n)
    U_new = np.zeros((T, n))
    costs = np.zeros(K)
    noise = np.zeros((K, T, n)) if want_noise else None
    st = lib().ora_update(C.byref(rb), C.byref(c), C.byref(tg), _p(_vec(q0, n)),
                          _p(_vec(qd0, n)), _p(U), C.c_uint64(seed), C.c_uint64(tick),
                          _p(U_new), _p(costs), _p(noise) if noise is not None else None,
                          int(nthreads))
    return st, U_new, costs, noise


def warm_start(U, s):
    """Warm start after s horizon steps (ora_warm_start)."""
    U = np.ascontiguousarray(U, dtype=np.float64)
    T, n = U.shape
    out = np.zeros((T, n))
    lib().ora_warm_start(int(T), int(n), _p(U.ravel()), float(s), _p(out))
    return out


def plant_step(robot, cost, q, qd, u, dt, substeps):
    rb, c = robot_struct(robot), cost_struct(cost)
    q = _vec(q, rb.n).copy()
    qd = _vec(qd, rb.n).copy()
    lib().ora_plant_step(C.byref(rb), C.byref(c), _p(q), _p(qd), _p(_vec(u, rb.n)),
                         float(dt), int(substeps))
    return q, qd


def max_threads():
    return int(lib().ora_max_threads())
