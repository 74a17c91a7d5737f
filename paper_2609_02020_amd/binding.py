"""Thin Python binding of libmppi.so (the C ABI declared in include/mppi.h).

Argument marshalling only: every step of the update runs in the library's
HIP kernels.  PyTorch is used for device memory and streams (tensors are
passed by ``data_ptr()``).  If the compiled library is missing the import
of a solver fails with an error; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmppi.so")
NJ = 7

OK, EINVAL, ENONFINITE, ENOMEM, EDEVICE, ENOTSUP, ESCRATCH = range(7)
FP32, FP64 = 0, 1
EXT_NONE, EXT_CONST, EXT_WALL = 0, 1, 2


class MppiError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s failed: %s (status %d)" % (what, strerror(status), status))
        self.status = status


class LinkParams(C.Structure):
    _fields_ = [("R_parent", C.c_double * 9), ("r_parent", C.c_double * 3),
                ("mass", C.c_double), ("com", C.c_double * 3),
                ("inertia_com", C.c_double * 6), ("armature", C.c_double),
                ("q_min", C.c_double), ("q_max", C.c_double),
                ("qd_max", C.c_double), ("tau_max", C.c_double)]


class RobotParams(C.Structure):
    _fields_ = [("n_joints", C.c_int), ("link", LinkParams * NJ),
                ("R_ee", C.c_double * 9), ("r_ee", C.c_double * 3),
                ("gravity", C.c_double * 3)]


MAX_OBSTACLES, MAX_PAIRS = 4, 32
DYN_ABA, DYN_EXPLICIT_M = 0, 1


class CostParams(C.Structure):
    _fields_ = [("K", C.c_int), ("T", C.c_int), ("dt", C.c_double),
                ("lam", C.c_double), ("sigma", C.c_double * NJ),
                ("W_pos", C.c_double * 3), ("W_ori", C.c_double * 3),
                ("W_force", C.c_double * 6), ("W_reg", C.c_double * 6),
                ("w_q", C.c_double), ("w_qd", C.c_double), ("w_tau", C.c_double),
                ("w_post", C.c_double), ("q_rest", C.c_double * NJ),
                ("w_terminal", C.c_double), ("force_mode", C.c_int),
                ("ext_mode", C.c_int), ("F_ext", C.c_double * 6),
                ("wall_n", C.c_double * 3), ("wall_d0", C.c_double),
                ("wall_k", C.c_double), ("wall_c", C.c_double),
                ("precision", C.c_int), ("lambda_fp64_threshold", C.c_double),
                ("w_collision", C.c_double), ("n_obstacles", C.c_int),
                ("obstacles", (C.c_double * 6) * MAX_OBSTACLES), ("n_pairs", C.c_int),
                ("pairs", (C.c_int * 2) * MAX_PAIRS), ("d_th", C.c_double * MAX_PAIRS),
                ("dynamics", C.c_int), ("noise_rho", C.c_double), ("iterations", C.c_int)]


class Target(C.Structure):
    _fields_ = [("p_des", C.c_double * 3), ("quat_des", C.c_double * 4),
                ("F_des", C.c_double * 6)]


class DeviceIO(C.Structure):
    _fields_ = [("q", C.c_void_p), ("qd", C.c_void_p), ("target", C.c_void_p),
                ("U_nominal", C.c_void_p), ("U_new", C.c_void_p), ("U_shift", C.c_void_p),
                ("costs", C.c_void_p), ("noise", C.c_void_p), ("status", C.c_void_p),
                ("seed", C.c_uint64), ("tick", C.c_uint64)]


def _fill(arr, values):
    vals = np.asarray(values, dtype=np.float64).ravel()
    if vals.size != len(arr):
        raise ValueError("expected %d values, got %d" % (len(arr), vals.size))
    for i, v in enumerate(vals):
        arr[i] = float(v)


def robot_params(robot: dict) -> RobotParams:
    rp = RobotParams()
    rp.n_joints = int(robot["n"])
    if rp.n_joints != NJ or len(robot["links"]) != NJ:
        raise ValueError("the kernels are built for %d joints" % NJ)
    for i, L in enumerate(robot["links"]):
        d = rp.link[i]
        _fill(d.R_parent, L["R_parent"])
        _fill(d.r_parent, L["r_parent"])
        d.mass = float(L["mass"])
        _fill(d.com, L["com"])
        _fill(d.inertia_com, L["inertia"])
        d.armature = float(L["armature"])
        d.q_min, d.q_max = float(L["q_min"]), float(L["q_max"])
        d.qd_max, d.tau_max = float(L["qd_max"]), float(L["tau_max"])
    _fill(rp.R_ee, robot["R_ee"])
    _fill(rp.r_ee, robot["r_ee"])
    _fill(rp.gravity, robot.get("gravity", [0.0, 0.0, -9.81]))
    return rp


def cost_params(cost: dict, precision: int = FP32, lambda_fp64_threshold: float = 0.05) -> CostParams:
    cp = CostParams()
    cp.K, cp.T = int(cost["K"]), int(cost["T"])
    cp.dt, cp.lam = float(cost["dt"]), float(cost["lambda"])
    _fill(cp.sigma, cost["sigma"])
    for key in ("W_pos", "W_ori", "W_force", "W_reg", "q_rest", "F_ext", "wall_n"):
        _fill(getattr(cp, key), cost.get(key, [0.0] * len(getattr(cp, key))))
    for key in ("w_q", "w_qd", "w_tau", "w_post", "wall_d0", "wall_k", "wall_c"):
        setattr(cp, key, float(cost.get(key, 0.0)))
    cp.w_terminal = float(cost.get("w_terminal", 1.0))
    cp.force_mode = int(cost.get("force_mode", 0))
    cp.ext_mode = int(cost.get("ext_mode", EXT_NONE))
    cp.precision = int(precision)
    cp.lambda_fp64_threshold = float(lambda_fp64_threshold)
    cp.w_collision = float(cost.get("w_collision", 0.0))
    obs, pairs = cost.get("obstacles", []), cost.get("pairs", [])
    if len(obs) > MAX_OBSTACLES or len(pairs) > MAX_PAIRS:
        raise ValueError("at most %d obstacles and %d collision pairs" % (MAX_OBSTACLES, MAX_PAIRS))
    cp.n_obstacles = len(obs)
    for o, seg in enumerate(obs):
        _fill(cp.obstacles[o], seg)
    cp.n_pairs = len(pairs)
    for i, (a, b) in enumerate(pairs):
        cp.pairs[i][0], cp.pairs[i][1] = int(a), int(b)
        cp.d_th[i] = float(cost["d_th"][i])
    cp.dynamics = int(cost.get("dynamics", DYN_ABA))
    cp.noise_rho = float(cost.get("noise_rho", 0.0))
    cp.iterations = int(cost.get("iterations", 1))
    return cp


def target_params(target: dict) -> Target:
    t = Target()
    _fill(t.p_des, target["p_des"])
    _fill(t.quat_des, target.get("quat_des", [1.0, 0.0, 0.0, 0.0]))
    _fill(t.F_des, target.get("F_des", [0.0] * 6))
    return t


def target_vector(target: dict) -> np.ndarray:
    """The 13-double device layout: p_des[3], quat_des[4], F_des[6]."""
    return np.concatenate([np.asarray(target["p_des"], float),
                           np.asarray(target.get("quat_des", [1.0, 0.0, 0.0, 0.0]), float),
                           np.asarray(target.get("F_des", [0.0] * 6), float)])


_lib = None


def lib():
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same soname; loading it
        # first makes libmppi.so bind to that one instance, so device
        # pointers and streams from torch are valid in the library.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmppi.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P, vp = C.POINTER, C.c_void_p
        L.mppi_create.argtypes = [P(RobotParams), P(CostParams), P(vp)]
        L.mppi_destroy.argtypes = [vp]
        L.mppi_set_cost.argtypes = [vp, P(CostParams)]
        L.mppi_update.argtypes = [vp, P(C.c_double), P(C.c_double), P(Target), P(C.c_double),
                                  C.c_uint64, C.c_uint64, P(C.c_double), P(C.c_double)]
        L.mppi_update_async.argtypes = [vp, P(DeviceIO), vp]
        L.mppi_update_noalloc.argtypes = [P(RobotParams), P(CostParams), P(DeviceIO), vp]
        L.mppi_rollout_async.argtypes = [vp, P(DeviceIO), vp]
        L.mppi_weights_async.argtypes = [vp, P(DeviceIO), vp]
        L.mppi_plant_step_async.argtypes = [vp, vp, vp, vp, C.c_double, C.c_int, vp]
        L.mppi_plant_step_wrench_async.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_int, vp]
        L.mppi_ee_pose_async.argtypes = [vp, vp, C.c_int, vp, vp]
        L.mppi_warm_start_async.argtypes = [vp, vp, vp, C.c_double, vp]
        L.mppi_set_launch.argtypes = [vp, C.c_int]
        L.mppi_autotune.argtypes = [vp, P(DeviceIO), C.c_int, vp, P(C.c_int), P(C.c_float)]
        L.mppi_set_autotune_cache.argtypes = [C.c_char_p]
        L.mppi_select_nominal_async.argtypes = [vp, P(DeviceIO), vp, vp, vp]
        L.mppi_strerror.argtypes = [C.c_int]
        L.mppi_strerror.restype = C.c_char_p
        L.mppi_version.restype = C.c_char_p
        _lib = L
    return _lib


def set_autotune_cache(path):
    """Autotune cache file of both tuners (mppi_set_autotune_cache); None: off."""
    st = lib().mppi_set_autotune_cache(None if path is None else str(path).encode())
    if st:
        raise MppiError(st, "mppi_set_autotune_cache")


def strerror(status: int) -> str:
    try:
        return lib().mppi_strerror(int(status)).decode()
    except ImportError:
        return "status %d" % status


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _dev(t, dtype: str, n: int, name: str):
    """Device pointer of a torch tensor that a kernel reads or writes n
    elements of, after checking what the C ABI cannot check on a raw
    pointer: a CUDA (HIP) tensor, contiguous, of the element type the
    kernels use, with at least n elements.  None passes through (the
    library decides whether the argument is optional)."""
    if t is None:
        return None
    import torch
    if not getattr(t, "is_cuda", False):
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.dtype != getattr(torch, dtype):
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.numel() < n:
        raise ValueError("%s needs %d elements, got %d" % (name, n, t.numel()))
    return C.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        return None
    return C.c_void_p(int(stream.cuda_stream))


def _device_io(io: dict, K: int, T: int, precision: int) -> DeviceIO:
    """mppi_device_io of one update from a dict of torch device tensors,
    each checked against what the kernels read and write."""
    d = DeviceIO()
    rdt = "float64" if precision == FP64 else "float32"
    TJ = T * NJ
    spec = {"q": ("float64", NJ), "qd": ("float64", NJ), "target": ("float64", 13),
            "U_nominal": ("float64", TJ), "U_new": ("float64", TJ), "U_shift": ("float64", TJ),
            "costs": (rdt, K), "noise": (rdt, TJ * K), "status": ("int32", 1)}
    for key, (dt, n) in spec.items():
        setattr(d, key, _dev(io.get(key), dt, n, key))
    d.seed = int(io.get("seed", 0))
    d.tick = int(io.get("tick", 0))
    return d


def update_noalloc(robot: dict, cost: dict, io: dict, precision: int = FP32,
                   lambda_fp64_threshold: float = 0.05, stream=None):
    """One update without a handle and without any allocation
    (mppi_update_noalloc): io as for Solver.update_async."""
    L = lib()
    rp = robot_params(robot)
    cp = cost_params(cost, precision, lambda_fp64_threshold)
    d = _device_io(io, cp.K, cp.T, precision)
    st = L.mppi_update_noalloc(C.byref(rp), C.byref(cp), C.byref(d), _stream_ptr(stream))
    if st:
        raise MppiError(st, "mppi_update_noalloc")


class Solver:
    """One MPPI problem: mppi_create / mppi_update / mppi_destroy."""

    def __init__(self, robot: dict, cost: dict, precision: int = FP32,
                 lambda_fp64_threshold: float = 0.05):
        self._lib = lib()
        self.K, self.T = int(cost["K"]), int(cost["T"])
        self.precision = precision
        self._h = C.c_void_p()
        self._rp = robot_params(robot)
        self._cp = cost_params(cost, precision, lambda_fp64_threshold)
        st = self._lib.mppi_create(C.byref(self._rp), C.byref(self._cp), C.byref(self._h))
        if st:
            raise MppiError(st, "mppi_create")

    def close(self):
        if self._h:
            self._lib.mppi_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_cost(self, cost: dict, lambda_fp64_threshold: float = 0.05):
        self._cp = cost_params(cost, self.precision, lambda_fp64_threshold)
        st = self._lib.mppi_set_cost(self._h, C.byref(self._cp))
        if st:
            raise MppiError(st, "mppi_set_cost")

    def update(self, q, qd, target: dict, U_nominal, seed: int, tick: int, want_costs=True):
        """Host-memory update.  Returns (status, U_new [T,7], costs [K] or None)."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        qd = np.ascontiguousarray(qd, dtype=np.float64)
        U = np.ascontiguousarray(U_nominal, dtype=np.float64).reshape(self.T, NJ)
        out = np.empty((self.T, NJ))
        costs = np.empty(self.K) if want_costs else None
        tg = target_params(target)
        st = self._lib.mppi_update(self._h, _dp(q), _dp(qd), C.byref(tg), _dp(U),
                                   C.c_uint64(seed), C.c_uint64(tick), _dp(out),
                                   _dp(costs) if costs is not None else None)
        if st not in (OK, ENONFINITE):
            raise MppiError(st, "mppi_update")
        return st, out, costs

    def _io(self, io: dict) -> DeviceIO:
        return _device_io(io, self.K, self.T, self.precision)

    def update_async(self, io: dict, stream=None):
        """Device update; io holds torch CUDA tensors (see mppi_device_io)."""
        d = self._io(io)
        st = self._lib.mppi_update_async(self._h, C.byref(d), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_update_async")

    def rollout_async(self, io: dict, stream=None):
        d = self._io(io)
        st = self._lib.mppi_rollout_async(self._h, C.byref(d), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_rollout_async")

    def weights_async(self, io: dict, stream=None):
        d = self._io(io)
        st = self._lib.mppi_weights_async(self._h, C.byref(d), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_weights_async")

    def plant_step_async(self, q, qd, u, dt: float, substeps: int, stream=None, wrench=None):
        """FP64 plant step (mppi_plant_step_async); with `wrench` (device
        [6] float64) a further world wrench at the EE point
        (mppi_plant_step_wrench_async)."""
        st = self._lib.mppi_plant_step_wrench_async(self._h, _dev(q, "float64", NJ, "q"),
                                                    _dev(qd, "float64", NJ, "qd"), _dev(u, "float64", NJ, "u"),
                                                    _dev(wrench, "float64", 6, "wrench"), float(dt), int(substeps),
                                                    _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_plant_step_wrench_async")

    def ee_pose_async(self, q, pose, stream=None):
        """EE position and quaternion (w >= 0) of the states q [n][7] into
        pose [n][7] (mppi_ee_pose_async); device float64 tensors."""
        n = q.numel() // NJ
        st = self._lib.mppi_ee_pose_async(self._h, _dev(q, "float64", n * NJ, "q"), int(n),
                                          _dev(pose, "float64", n * 7, "pose"), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_ee_pose_async")

    def autotune(self, io: dict, budget_ms: int = 30, stream=None):
        """Times launch shapes 8, 2 and 1 on io (mppi_autotune), keeps the
        fastest; returns (shape, [times in ms, -1 when taken from the cache])."""
        d = self._io(io)
        best = C.c_int()
        times = (C.c_float * 3)()
        st = self._lib.mppi_autotune(self._h, C.byref(d), int(budget_ms), _stream_ptr(stream), C.byref(best), times)
        if st:
            raise MppiError(st, "mppi_autotune")
        return best.value, list(times)

    def set_launch(self, waves_per_group: int):
        """Launch shape of the updates (mppi_set_launch): 1 or 2 waves per 64
        samples, or 8 lanes per sample."""
        st = self._lib.mppi_set_launch(self._h, int(waves_per_group))
        if st:
            raise MppiError(st, "mppi_set_launch")

    def warm_start_async(self, U_new, U_out, shift_steps: float, stream=None):
        """U_out = U_new advanced by shift_steps horizon steps (mppi_warm_start_async)."""
        TJ = self.T * NJ
        st = self._lib.mppi_warm_start_async(self._h, _dev(U_new, "float64", TJ, "U_new"),
                                             _dev(U_out, "float64", TJ, "U_out"), float(shift_steps),
                                             _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_warm_start_async")

    def select_nominal_async(self, io: dict, U_candidate, costs=None, stream=None):
        """Keeps io["U_nominal"] or replaces it with U_candidate, whichever
        has the lower noise-free rollout cost (mppi_select_nominal_async)."""
        d = self._io(io)
        st = self._lib.mppi_select_nominal_async(self._h, C.byref(d), _dev(U_candidate, "float64", self.T * NJ,
                                                                           "U_candidate"),
                                                 _dev(costs, "float64", 2, "costs"), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_select_nominal_async")


class ProblemDesc(C.Structure):
    _fields_ = [("robot", C.POINTER(RobotParams)), ("cost", C.POINTER(CostParams))]


class BatchIO(C.Structure):
    _fields_ = [("q", C.c_void_p), ("qd", C.c_void_p), ("target", C.c_void_p),
                ("U_nominal", C.c_void_p), ("U_new", C.c_void_p), ("U_shift", C.c_void_p),
                ("costs", C.c_void_p), ("status", C.c_void_p), ("seed", C.c_void_p)]


def _batch_lib():
    L = lib()
    if not hasattr(L, "_batch_ready"):
        P, vp = C.POINTER, C.c_void_p
        L.mppi_batch_create.argtypes = [P(ProblemDesc), C.c_int, P(vp)]
        L.mppi_batch_destroy.argtypes = [vp]
        L.mppi_batch_layout.argtypes = [vp, P(C.c_size_t), P(C.c_size_t), P(C.c_size_t), P(C.c_size_t)]
        L.mppi_batch_update_async.argtypes = [vp, P(BatchIO), C.c_uint64, vp]
        L.mppi_batch_set_launch.argtypes = [vp, C.c_int, C.c_int]
        L.mppi_batch_autotune.argtypes = [vp, P(BatchIO), C.c_int, vp, P(C.c_int), P(C.c_int),
                                          P(C.c_float)]
        L.mppi_batch_graph_capture.argtypes = [vp, P(BatchIO)]
        L.mppi_batch_set_tick.argtypes = [vp, C.c_uint64]
        L.mppi_batch_graph_launch.argtypes = [vp, vp]
        L.mppi_batch_plant_step_async.argtypes = [vp, P(BatchIO), C.c_double, C.c_int, vp]
        L.mppi_batch_warm_start_async.argtypes = [vp, vp, vp, C.c_double, vp]
        L.mppi_batch_select_nominal_async.argtypes = [vp, P(BatchIO), vp, vp, vp]
        L._batch_ready = True
    return L


class Batch:
    """Many independent MPPI problems in one persistent launch
    (mppi_batch_*).  Problems are (robot dict, cost dict) pairs; rollouts
    run in FP32."""

    def __init__(self, problems, lambda_fp64_threshold: float = 0.05):
        self._lib = _batch_lib()
        self.n = len(problems)
        self._rps = [robot_params(r) for r, _ in problems]
        self._cps = [cost_params(c, FP32, lambda_fp64_threshold) for _, c in problems]
        self.K = [int(c["K"]) for _, c in problems]
        self.T = [int(c["T"]) for _, c in problems]
        descs = (ProblemDesc * self.n)()
        for i in range(self.n):
            descs[i].robot = C.pointer(self._rps[i])
            descs[i].cost = C.pointer(self._cps[i])
        self._h = C.c_void_p()
        st = self._lib.mppi_batch_create(descs, self.n, C.byref(self._h))
        if st:
            raise MppiError(st, "mppi_batch_create")
        u_off = (C.c_size_t * self.n)()
        k_off = (C.c_size_t * self.n)()
        ut, kt = C.c_size_t(), C.c_size_t()
        self._lib.mppi_batch_layout(self._h, u_off, k_off, C.byref(ut), C.byref(kt))
        self.u_off, self.k_off = list(u_off), list(k_off)
        self.u_total, self.k_total = ut.value, kt.value

    def close(self):
        if self._h:
            self._lib.mppi_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _io(self, io: dict) -> BatchIO:
        d = BatchIO()
        n = self.n
        spec = {"q": ("float64", n * NJ), "qd": ("float64", n * NJ), "target": ("float64", n * 13),
                "U_nominal": ("float64", self.u_total), "U_new": ("float64", self.u_total),
                "U_shift": ("float64", self.u_total), "costs": ("float32", self.k_total),
                "status": ("int32", n), "seed": ("int64", n)}
        for key, (dt, cnt) in spec.items():
            setattr(d, key, _dev(io.get(key), dt, cnt, key))
        return d

    def update_async(self, io: dict, tick: int, stream=None):
        d = self._io(io)
        st = self._lib.mppi_batch_update_async(self._h, C.byref(d), C.c_uint64(tick), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_batch_update_async")

    def set_launch(self, waves_per_group: int, groups: int):
        st = self._lib.mppi_batch_set_launch(self._h, int(waves_per_group), int(groups))
        if st:
            raise MppiError(st, "mppi_batch_set_launch")

    def autotune(self, io: dict, reps: int = 3, stream=None):
        d = self._io(io)
        w, g = C.c_int(), C.c_int()
        times = (C.c_float * 16)()
        st = self._lib.mppi_batch_autotune(self._h, C.byref(d), int(reps), _stream_ptr(stream),
                                           C.byref(w), C.byref(g), times)
        if st:
            raise MppiError(st, "mppi_batch_autotune")
        return w.value, g.value, list(times)

    def graph_capture(self, io: dict):
        self._graph_io = self._io(io)
        st = self._lib.mppi_batch_graph_capture(self._h, C.byref(self._graph_io))
        if st:
            raise MppiError(st, "mppi_batch_graph_capture")

    def set_tick(self, tick: int):
        st = self._lib.mppi_batch_set_tick(self._h, C.c_uint64(tick))
        if st:
            raise MppiError(st, "mppi_batch_set_tick")

    def graph_launch(self, stream=None):
        st = self._lib.mppi_batch_graph_launch(self._h, _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_batch_graph_launch")

    def plant_step_async(self, io: dict, dt: float, substeps: int, stream=None):
        """Advances io["q"], io["qd"] of every problem by the FP64 plant,
        holding the first row of its U_new."""
        d = self._io(io)
        st = self._lib.mppi_batch_plant_step_async(self._h, C.byref(d), float(dt), int(substeps),
                                                   _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_batch_plant_step_async")

    def warm_start_async(self, U_new, U_out, shift_steps: float, stream=None):
        """Packed U_out = U_new advanced by shift_steps horizon steps."""
        st = self._lib.mppi_batch_warm_start_async(self._h, _dev(U_new, "float64", self.u_total, "U_new"),
                                                   _dev(U_out, "float64", self.u_total, "U_out"),
                                                   float(shift_steps), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_batch_warm_start_async")

    def select_nominal_async(self, io: dict, U_candidates, costs=None, stream=None):
        d = self._io(io)
        st = self._lib.mppi_batch_select_nominal_async(self._h, C.byref(d),
                                                       _dev(U_candidates, "float64", self.u_total, "U_candidates"),
                                                       _dev(costs, "float64", 2 * self.n, "costs"),
                                                       _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_batch_select_nominal_async")


MLP_INPUTS, MLP_OUTPUTS, MLP_PARAMS = 21, 126, 169598


class AdamParams(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double)]


def _mlp_lib():
    L = lib()
    if not hasattr(L, "_mlp_ready"):
        P, vp = C.POINTER, C.c_void_p
        L.mppi_mlp_create.argtypes = [P(RobotParams), C.c_int, P(vp)]
        L.mppi_mlp_destroy.argtypes = [vp]
        L.mppi_mlp_set_params.argtypes = [vp, P(C.c_float), C.c_size_t]
        L.mppi_mlp_get_params.argtypes = [vp, P(C.c_float), C.c_size_t]
        L.mppi_mlp_forward_async.argtypes = [vp, vp, C.c_int, vp, vp]
        L.mppi_mlp_grad_async.argtypes = [vp, vp, vp, C.c_int, vp, vp, vp]
        L.mppi_mlp_adam_async.argtypes = [vp, P(AdamParams), vp]
        L.mppi_mlp_train_step_async.argtypes = [vp, vp, vp, C.c_int, P(AdamParams), vp, vp]
        L.mppi_mlp_propose_async.argtypes = [vp, C.c_int, vp, vp, vp, vp, C.c_int, vp]
        L.mppi_mlp_encode_async.argtypes = [vp, C.c_int, vp, vp, vp, vp, C.c_int, vp, vp, vp]
        L._mlp_ready = True
    return L


class Mlp:
    """The learned proposal network (mppi_mlp_*).  Device arrays are torch
    CUDA tensors (float32 rows of 21 inputs / 126 outputs; float64 states)."""

    def __init__(self, robot: dict, max_batch: int):
        self._lib = _mlp_lib()
        self._rp = robot_params(robot)
        self.max_batch = int(max_batch)
        self._h = C.c_void_p()
        st = self._lib.mppi_mlp_create(C.byref(self._rp), self.max_batch, C.byref(self._h))
        if st:
            raise MppiError(st, "mppi_mlp_create")

    def close(self):
        if self._h:
            self._lib.mppi_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, theta):
        a = np.ascontiguousarray(theta, dtype=np.float32)
        st = self._lib.mppi_mlp_set_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size)
        if st:
            raise MppiError(st, "mppi_mlp_set_params")

    def get_params(self) -> np.ndarray:
        a = np.empty(MLP_PARAMS, dtype=np.float32)
        st = self._lib.mppi_mlp_get_params(self._h, a.ctypes.data_as(C.POINTER(C.c_float)), a.size)
        if st:
            raise MppiError(st, "mppi_mlp_get_params")
        return a

    def _rows(self, x):
        B = int(x.shape[0])
        if x.dim() != 2 or x.shape[1] != MLP_INPUTS:
            raise ValueError("x must be [B][%d]" % MLP_INPUTS)
        return B

    def forward_async(self, x, y, stream=None):
        B = self._rows(x)
        st = self._lib.mppi_mlp_forward_async(self._h, _dev(x, "float32", B * MLP_INPUTS, "x"), B,
                                              _dev(y, "float32", B * MLP_OUTPUTS, "y"), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_mlp_forward_async")

    def grad_async(self, x, y_target, grad=None, loss=None, stream=None):
        B = self._rows(x)
        st = self._lib.mppi_mlp_grad_async(self._h, _dev(x, "float32", B * MLP_INPUTS, "x"),
                                           _dev(y_target, "float32", B * MLP_OUTPUTS, "y_target"), B,
                                           _dev(grad, "float32", MLP_PARAMS, "grad"), _dev(loss, "float32", 1, "loss"),
                                           _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_mlp_grad_async")

    @staticmethod
    def _adam(lr, beta1, beta2, eps):
        return AdamParams(float(lr), float(beta1), float(beta2), float(eps))

    def adam_async(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        p = self._adam(lr, beta1, beta2, eps)
        st = self._lib.mppi_mlp_adam_async(self._h, C.byref(p), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_mlp_adam_async")

    def train_step_async(self, x, y_target, loss=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        p = self._adam(lr, beta1, beta2, eps)
        B = self._rows(x)
        st = self._lib.mppi_mlp_train_step_async(self._h, _dev(x, "float32", B * MLP_INPUTS, "x"),
                                                 _dev(y_target, "float32", B * MLP_OUTPUTS, "y_target"), B,
                                                 C.byref(p), _dev(loss, "float32", 1, "loss"), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_mlp_train_step_async")

    def propose_async(self, q, qd, target, U, u_stride=MLP_OUTPUTS, stream=None):
        n = int(q.shape[0])
        if u_stride < MLP_OUTPUTS:
            raise ValueError("u_stride must be at least %d" % MLP_OUTPUTS)
        st = self._lib.mppi_mlp_propose_async(self._h, n, _dev(q, "float64", n * NJ, "q"),
                                              _dev(qd, "float64", n * NJ, "qd"),
                                              _dev(target, "float64", n * 13, "target"),
                                              _dev(U, "float64", (n - 1) * u_stride + MLP_OUTPUTS, "U"),
                                              int(u_stride), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_mlp_propose_async")

    def encode_async(self, q, qd, target, x, U=None, y=None, u_stride=MLP_OUTPUTS, stream=None):
        """Training rows: features x [n][21] and, with U and y, the
        normalised targets y [n][126] = U / tau_max."""
        n = int(q.shape[0])
        if u_stride < MLP_OUTPUTS:
            raise ValueError("u_stride must be at least %d" % MLP_OUTPUTS)
        st = self._lib.mppi_mlp_encode_async(self._h, n, _dev(q, "float64", n * NJ, "q"),
                                             _dev(qd, "float64", n * NJ, "qd"),
                                             _dev(target, "float64", n * 13, "target"),
                                             _dev(U, "float64", (n - 1) * u_stride + MLP_OUTPUTS, "U"),
                                             int(u_stride), _dev(x, "float32", n * MLP_INPUTS, "x"),
                                             _dev(y, "float32", n * MLP_OUTPUTS, "y"), _stream_ptr(stream))
        if st:
            raise MppiError(st, "mppi_mlp_encode_async")
