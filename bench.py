"""Benchmark: MPPI update rate and ABA rollout steps/s on one MI355X.

A step is one MPPI update of the contact workload (K=4096 samples, T=18
steps, dt=0.01 s, 7-DoF arm, FP32 rollouts) on the default launch shape:
the eight-lanes-per-sample rollout kernel (Philox noise, forward dynamics
from composite-rigid-body inertias and an LDL^T solve, force estimate,
cost, Euler step, per-workgroup partials of Eq. 4) and its merge launch
(minimum-shifted exponentiated weights, weighted noise sum, shifted warm
start), with every input resident in HBM.  The articulated-body launches
(one and two waves per 64 samples) are timed beside it, and the fastest of
them gives aba_rollout_steps_per_s.  Consecutive steps
chain the warm start (U_nominal <- shifted U_new) and advance the Philox
tick; the measured state is the one reached after the warm-up ticks of a
closed loop with the on-device plant.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MPPI update rate (Hz) + ABA rollout steps/s, K=4096 T=18 7-DoF, FP32"
# Algorithmic floating-point operations of one sample-step and of the
# per-sample terminal cost: the work of the method on the articulated-body
# route (forward kinematics, articulated-body dynamics, the force estimate
# in its least-squares form, the cost and the Euler step), counted by
# running the per-lane kernels' per-sample code with an op-counting scalar
# (tests/opcount.cpp; add, mul, div, sqrt = 1 flop each, a fused
# multiply-add = 2).  Every launch shape and route is credited with this
# same work per sample-step; the eight-lane default computes the same
# quantities by the composite-rigid-body route and executes more
# instructions for them (every lane factorises M).  Contact workload
# (force estimate, wall, orientation cost on).
FLOPS_PER_SAMPLE_STEP = 6475
FLOPS_PER_SAMPLE_TERMINAL = 822
# Free-space problems (no wall, no force term, no orientation cost).
FLOPS_PER_SAMPLE_STEP_FREE = 4573
FLOPS_PER_SAMPLE_TERMINAL_FREE = 704
# The paper's own dynamics route (M by Eq. 8, Cholesky), contact workload.
FLOPS_PER_SAMPLE_STEP_EXPLICIT = 6581
# Eq. 4b: one multiply-add per sample and output row (weighted noise sum).
FLOPS_PER_SAMPLE_ROW_WEIGHT = 2
FP32_PEAK_TFLOPS = 157.3          # MI355X vector FP32 (AMD published)

# HBM bytes per launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs of this
# script, each scaled by what the counter reads for a plain device copy of
# known size (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000 on gfx950), taken on the
# kernel sources whose digest is recorded here; reported as null once the
# sources differ.
PROFILED_DIGEST = "9389df91679e6d76"
PROFILED_TRAFFIC = {"update_group_kernel": 340034 + 159744 + 476486 + 1956,   # K=4096, T=18 contact workload:
                                                            # the group kernel and its merge launch
                    # 64-problem batch, per launch shape the autotuner may pick (waves per
                    # group x groups); the one-lane shapes mostly register-spill stores
                    "batch_kernel_w1x2048": 106361459 + 324806144,
                    "batch_kernel_w2x1024": 118716882 + 352157440,
                    "batch_kernel_w4x512": 104396139 + 333902592,
                    "batch_kernel_w8x256": 5992043 + 10652006,    # eight lanes per sample
                    "mlp_train": 5863884 + 1737728 + 4833908 + 678432}   # forward/backward + weight
                                                                          # gradients, 512 rows


def kernel_source_digest():
    """SHA-256 (16 hex digits) over the HIP sources and the C-ABI header."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2609_02020_amd", "csrc")
    files = [os.path.join(d, n) for n in sorted(os.listdir(d)) if n.endswith((".hip", ".hpp", ".h"))]
    for f in files + [os.path.join(ROOT, "include", "mppi.h")]:
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel):
    return PROFILED_TRAFFIC.get(kernel) if kernel_source_digest() == PROFILED_DIGEST else None


def span_ms(torch, stream, fn, n):
    """Mean GPU time per call of fn(i), i = 0..n-1, launched back to back:
    one pair of HIP events around all n calls (events around each call put
    their own packets between the launches, ~2 us of queue time per pair)."""
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for i in range(n):
        fn(i)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / n


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=300)
    p.add_argument("--warmup", type=int, default=30)
    p.add_argument("--workload", default="wall_k4096")
    p.add_argument("--case", type=int, default=0)
    p.add_argument("--cpu-seconds", type=float, default=12.0,
                   help="budget of the oracle CPU-baseline sample")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--batch-ticks", type=int, default=30,
                   help="graph replays of the 64-problem batched tick (0: skip)")
    p.add_argument("--no-mlp", action="store_true", help="skip the proposal-network timings")
    p.add_argument("--cpu-study", type=float, default=0.0, metavar="SECONDS",
                   help="only time the oracle (no GPU): the single-update, contact and precision "
                        "workloads on one thread and on every core, SECONDS each, one JSON line")
    p.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                   help="after the timed region, copy a MIB-sized buffer 5 times (a plain copy "
                        "kernel of known size, to calibrate HBM byte counters)")
    return p.parse_args()


def cpu_baseline(case, budget_s):
    """The FP64 CPU oracle, as it stands, on the host cores: full updates of
    the same workload (same K, T, seeds) until the time budget is used."""
    from oracle import oracle as ora
    ora.build()
    n, t0 = 0, time.perf_counter()
    while True:
        ora.update(case["robot"], case["cost"], case["target"], case["q0"], case["qd0"],
                   case["U_nom"], case["seed"], n, want_noise=False)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 1000:
            break
    K, T = case["cost"]["K"], case["cost"]["T"]
    return {"value": n / el, "unit": "Hz", "cores": ora.max_threads(), "kind": "oracle",
            "sample": "%d full oracle updates (K=%d, T=%d, FP64, OpenMP over samples) in %.1f s; "
                      "%.3g sample-steps/s" % (n, K, T, el, n * K * T / el),
            "cpu": cpu_model()}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_study(budget_s):
    """The oracle's update rate and sample-steps/s on one thread and on all
    cores for the single-update (K=256, T=18, position cost), contact
    (K=4096, T=18) and precision (K=16384, T=36) workloads."""
    from oracle import oracle as ora
    from paper_2609_02020_amd import inputs
    ora.build()
    W = inputs.load()
    rows = []
    for name in ("single_k256", "wall_k4096", "precision_k16384"):
        case = W[name][0]
        K, T = case["cost"]["K"], case["cost"]["T"]
        for threads in (1, ora.max_threads()):
            n, t0 = 0, time.perf_counter()
            while True:
                ora.update(case["robot"], case["cost"], case["target"], case["q0"], case["qd0"], case["U_nom"],
                           case["seed"], n, nthreads=threads, want_noise=False)
                n += 1
                el = time.perf_counter() - t0
                if el >= budget_s:
                    break
            rows.append({"workload": "%s[0]" % name, "K": K, "T": T, "threads": threads, "updates": n,
                         "seconds": el, "updates_per_s": n / el, "sample_steps_per_s": n * K * T / el})
    return {"cpu": cpu_model(), "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "rows": rows}


# Proposal network 21-256-256-256-126 (unpadded dimensions): a forward
# pass is 2 * 168,704 flops per row; training adds the backward products of
# layers 4..2 (2 * 163,328) and the weight gradients (2 * 168,704).
MLP_FWD_FLOPS_PER_ROW = 2 * (21 * 256 + 256 * 256 + 256 * 256 + 256 * 126)
MLP_TRAIN_FLOPS_PER_ROW = MLP_FWD_FLOPS_PER_ROW + 2 * (126 * 256 + 256 * 256 + 256 * 256) + MLP_FWD_FLOPS_PER_ROW
BF16_MFMA_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix cores (AMD published)


def mlp_bench(B, inputs, robot, torch, dev, reps=50, rows=512):
    """The proposal network's kernels: one training step (forward, MSE,
    backward, weight gradients, Adam) on a batch of `rows` synthetic rows,
    and the proposal (features, forward, torque scaling) for 1 and 64
    states, each timed with HIP events over `reps` launches."""
    import numpy as np
    net = B.Mlp(robot, max(rows, 64))
    net.set_params(inputs.draw_mlp_params(1).astype(np.float32))
    X, Y = inputs.draw_mlp_batch(2, rows)
    Xd = torch.tensor(X, dtype=torch.float32, device=dev)
    Yd = torch.tensor(Y, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(5):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    loss = torch.zeros(1, device=dev)
    grad_ms = timed(lambda: net.grad_async(Xd, Yd, loss=loss, stream=stream))
    train_ms = timed(lambda: net.train_step_async(Xd, Yd, loss, lr=1e-4, stream=stream))
    fwd_ms = timed(lambda: net.forward_async(Xd, torch.empty((rows, 126), device=dev), stream=stream))
    prop = {}
    for n in (1, 64):
        q = torch.zeros((n, 7), dtype=torch.float64, device=dev)
        tg = torch.zeros((n, 13), dtype=torch.float64, device=dev)
        tg[:, 3] = 1.0
        U = torch.empty((n, 126), dtype=torch.float64, device=dev)
        prop[n] = timed(lambda: net.propose_async(q, q, tg, U, stream=stream))
    net.close()
    # the same training step on a batch that gives every CU a workgroup
    big = 4096
    net = B.Mlp(robot, big)
    net.set_params(inputs.draw_mlp_params(1).astype(np.float32))
    Xb, Yb = inputs.draw_mlp_batch(3, big)
    Xbd = torch.tensor(Xb, dtype=torch.float32, device=dev)
    Ybd = torch.tensor(Yb, dtype=torch.float32, device=dev)
    big_grad = timed(lambda: net.grad_async(Xbd, Ybd, loss=loss, stream=stream))
    big_train = timed(lambda: net.train_step_async(Xbd, Ybd, loss, lr=1e-4, stream=stream))
    net.close()
    big_tf = MLP_TRAIN_FLOPS_PER_ROW * big / (big_grad * 1e-3) / 1e12
    tf = MLP_TRAIN_FLOPS_PER_ROW * rows / (grad_ms * 1e-3) / 1e12
    return {"rows": rows, "train_step_ms": train_ms, "train_rows_per_s": rows / (train_ms * 1e-3),
            "batch_4096": {"grad_ms": big_grad, "train_step_ms": big_train,
                           "train_rows_per_s": big / (big_train * 1e-3), "grad_tflops": big_tf,
                           "grad_frac_of_bf16_peak": big_tf / BF16_MFMA_PEAK_TFLOPS},
            "grad_ms": grad_ms, "forward_ms": fwd_ms, "propose_us": {"1": 1e3 * prop[1], "64": 1e3 * prop[64]},
            "flops_per_row": {"forward": MLP_FWD_FLOPS_PER_ROW, "train": MLP_TRAIN_FLOPS_PER_ROW},
            "roofline": {"bound": "mfma", "achieved": tf, "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / BF16_MFMA_PEAK_TFLOPS, "traffic": profiled_traffic("mlp_train"),
                         "kernel": "mlp_forward_kernel<true> + mlp_wgrad_kernel (forward, backward, gradients)",
                         "flops_per_launch": MLP_TRAIN_FLOPS_PER_ROW * rows}}


def collision_bench(B, case, torch, dev, steps=100):
    """The contact workload with the collision term of Eqs. 14-15 (two
    obstacles, 20 pairs): device-resident updates timed with HIP events."""
    solver = B.Solver(case["robot"], case["cost"], B.FP32)
    f64 = dict(dtype=torch.float64, device=dev)
    K, T = case["cost"]["K"], case["cost"]["T"]
    io = {"q": torch.tensor(case["q0"], **f64), "qd": torch.tensor(case["qd0"], **f64),
          "target": torch.tensor(B.target_vector(case["target"]), **f64),
          "U_nominal": torch.tensor(case["U_nom"], **f64), "U_new": torch.empty((T, 7), **f64),
          "U_shift": torch.empty((T, 7), **f64), "costs": torch.empty(K, dtype=torch.float32, device=dev),
          "status": torch.zeros(1, dtype=torch.int32, device=dev), "seed": case["seed"], "tick": 0}
    stream = torch.cuda.current_stream()
    for i in range(10):
        io["tick"] = i
        solver.update_async(io, stream)

    def one(i):
        io["tick"] = 10 + i
        solver.update_async(io, stream)
    ms = span_ms(torch, stream, one, steps)
    solver.close()
    return {"workload": "collision_k4096[0]: the contact workload plus %d obstacles and %d collision pairs "
                        "(w_collision = %g), K=%d, T=%d" % (len(case["cost"]["obstacles"]), len(case["cost"]["pairs"]),
                                                          case["cost"]["w_collision"], K, T),
            "update_kernel_ms": ms, "update_hz_kernel_only": 1e3 / ms, "rollout_steps_per_s": K * T / (ms * 1e-3)}


def explicit_bench(B, case, torch, dev, steps=100):
    """The contact workload on both dynamics routes (articulated-body vs M
    by Eq. 8 with a Cholesky solve), both on the per-lane launch with one
    wave per 64 samples (the route of Eq. 8 has no eight-lane form):
    update-kernel time with HIP events."""
    f64 = dict(dtype=torch.float64, device=dev)
    K, T = case["cost"]["K"], case["cost"]["T"]
    res = {}
    for name, dyn in (("aba", B.DYN_ABA), ("explicit_m", B.DYN_EXPLICIT_M)):
        solver = B.Solver(case["robot"], dict(case["cost"], dynamics=dyn), B.FP32)
        solver.set_launch(1)
        io = {"q": torch.tensor(case["q0"], **f64), "qd": torch.tensor(case["qd0"], **f64),
              "target": torch.tensor(B.target_vector(case["target"]), **f64),
              "U_nominal": torch.tensor(case["U_nom"], **f64), "U_new": torch.empty((T, 7), **f64),
              "U_shift": torch.empty((T, 7), **f64), "costs": torch.empty(K, dtype=torch.float32, device=dev),
              "status": torch.zeros(1, dtype=torch.int32, device=dev), "seed": case["seed"], "tick": 0}
        stream = torch.cuda.current_stream()
        for i in range(10):
            io["tick"] = i
            solver.update_async(io, stream)

        def one(i):
            io["tick"] = 10 + i
            solver.update_async(io, stream)
        res[name + "_kernel_ms"] = span_ms(torch, stream, one, steps)
        solver.close()
    res["flops_per_sample_step"] = {"aba": FLOPS_PER_SAMPLE_STEP, "explicit_m": FLOPS_PER_SAMPLE_STEP_EXPLICIT}
    res["workload"] = "wall_k4096[0], K=%d, T=%d, FP32" % (K, T)
    res["launch"] = "one wave per 64 samples (per-lane kernels), both routes"
    return res


def sampling_bench(B, case, torch, dev, steps=100):
    """The contact workload with the sampling variants: independent draws,
    perturbations correlated in time (rho = 0.8) and three MPPI iterations
    per update (three fused launches): GPU time per update with HIP events."""
    f64 = dict(dtype=torch.float64, device=dev)
    K, T = case["cost"]["K"], case["cost"]["T"]
    res = {}
    for name, kw in (("iid", {}), ("ar1_rho0.8", {"noise_rho": 0.8}), ("iterations3", {"iterations": 3})):
        solver = B.Solver(case["robot"], dict(case["cost"], **kw), B.FP32)
        io = {"q": torch.tensor(case["q0"], **f64), "qd": torch.tensor(case["qd0"], **f64),
              "target": torch.tensor(B.target_vector(case["target"]), **f64),
              "U_nominal": torch.tensor(case["U_nom"], **f64), "U_new": torch.empty((T, 7), **f64),
              "U_shift": torch.empty((T, 7), **f64), "costs": torch.empty(K, dtype=torch.float32, device=dev),
              "status": torch.zeros(1, dtype=torch.int32, device=dev), "seed": case["seed"], "tick": 0}
        stream = torch.cuda.current_stream()
        for i in range(10):
            io["tick"] = i
            solver.update_async(io, stream)

        def one(i):
            io["tick"] = 10 + i
            solver.update_async(io, stream)
        res[name + "_update_ms"] = span_ms(torch, stream, one, steps)
        solver.close()
    res["workload"] = "wall_k4096[0], K=%d, T=%d, FP32" % (K, T)
    return res


def has_force(cost):
    return any(w != 0 for w in cost["W_force"]) or any(w != 0 for w in cost["W_reg"])


def problem_flops(cost):
    K, T = cost["K"], cost["T"]
    step, term = ((FLOPS_PER_SAMPLE_STEP, FLOPS_PER_SAMPLE_TERMINAL) if has_force(cost) else
                  (FLOPS_PER_SAMPLE_STEP_FREE, FLOPS_PER_SAMPLE_TERMINAL_FREE))
    return step * K * T + term * K + FLOPS_PER_SAMPLE_ROW_WEIGHT * K * T * 7


def batch_bench(B, cases, torch, dev, ticks):
    """64 independent problems (K in [512, 8192], T in [10, 50], half with
    the wall and force cost) per tick: one persistent launch, autotuned
    launch shape, replayed from a captured HIP graph.  The graph reads and
    advances its Philox tick on the device; the nominal sequences stay fixed
    across replays (each replay is a full update of all 64 problems)."""
    import numpy as np
    batch = B.Batch([(c["robot"], c["cost"]) for c in cases])
    f64 = dict(dtype=torch.float64, device=dev)
    U = np.zeros((batch.u_total // 7, 7))
    for p, c in enumerate(cases):
        U[batch.u_off[p] // 7: batch.u_off[p] // 7 + batch.T[p]] = np.asarray(c["U_nom"])[:batch.T[p]]
    io = {"q": torch.tensor(np.array([c["q0"] for c in cases]), **f64),
          "qd": torch.tensor(np.array([c["qd0"] for c in cases]), **f64),
          "target": torch.tensor(np.array([B.target_vector(c["target"]) for c in cases]), **f64),
          "U_nominal": torch.tensor(U, **f64), "U_new": torch.empty(U.shape, **f64),
          "U_shift": torch.empty(U.shape, **f64),
          "costs": torch.empty(batch.k_total, dtype=torch.float32, device=dev),
          "status": torch.zeros(len(cases), dtype=torch.int32, device=dev),
          "seed": torch.tensor([c["seed"] for c in cases], dtype=torch.int64, device=dev)}
    stream = torch.cuda.current_stream()
    wpg, groups, tune_ms = batch.autotune(io, reps=3, stream=stream)
    batch.graph_capture(io)
    batch.set_tick(0)
    for _ in range(3):
        batch.graph_launch(stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(ticks):
        batch.graph_launch(stream)
    b.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = io["status"].cpu().numpy()
    assert (st == B.OK).all(), st
    tick_ms = a.elapsed_time(b) / ticks
    sample_steps = sum(c["cost"]["K"] * c["cost"]["T"] for c in cases)
    flops = sum(problem_flops(c["cost"]) for c in cases)
    batch.close()
    return {"workload": "batch64: 64 problems, K in [%d, %d], T in [%d, %d], %d with the wall + force "
                        "cost, %d sample-steps per tick" % (
                            min(c["cost"]["K"] for c in cases), max(c["cost"]["K"] for c in cases),
                            min(c["cost"]["T"] for c in cases), max(c["cost"]["T"] for c in cases),
                            sum(has_force(c["cost"]) for c in cases), sample_steps),
            "ticks_per_s": ticks / elapsed, "tick_ms": tick_ms, "ticks": ticks,
            "problem_updates_per_s": len(cases) * ticks / elapsed,
            "rollout_steps_per_s": sample_steps / (tick_ms * 1e-3),
            "launch": {"waves_per_group": wpg, "groups": groups, "graph": True,
                       "lanes_per_sample": 8 if wpg == 8 else 1},
            "autotune_ms": {"%s_waves%d" % ("lanes8" if w == 8 else "wpg%d" % w, v): round(t, 4)
                            for (w, v), t in zip([(w, v) for w in (1, 2, 4, 8) for v in (256, 512, 1024, 2048)],
                                                 tune_ms)},
            "roofline": {"bound": "alu", "achieved": flops / (tick_ms * 1e-3) / 1e12,
                         "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": flops / (tick_ms * 1e-3) / 1e12 / FP32_PEAK_TFLOPS,
                         "traffic": profiled_traffic("batch_kernel_w%dx%d" % (wpg, groups)),
                         "kernel": "batch_group_kernel" if wpg == 8 else "batch_kernel",
                         "flops_per_launch": flops}}


def small_batch_bench(B, cases, torch, dev, reps=50):
    """A latency-bound batch (the first 8 problems of batch64 with K capped
    at 1024): the tick at one and at eight lanes per sample, each at the
    autotuner's best workgroup count for that lane count."""
    import numpy as np
    cases = [dict(c, cost=dict(c["cost"], K=min(c["cost"]["K"], 1024))) for c in cases[:8]]
    batch = B.Batch([(c["robot"], c["cost"]) for c in cases])
    f64 = dict(dtype=torch.float64, device=dev)
    U = np.zeros((batch.u_total // 7, 7))
    for p, c in enumerate(cases):
        U[batch.u_off[p] // 7: batch.u_off[p] // 7 + batch.T[p]] = np.asarray(c["U_nom"])[:batch.T[p]]
    io = {"q": torch.tensor(np.array([c["q0"] for c in cases]), **f64),
          "qd": torch.tensor(np.array([c["qd0"] for c in cases]), **f64),
          "target": torch.tensor(np.array([B.target_vector(c["target"]) for c in cases]), **f64),
          "U_nominal": torch.tensor(U, **f64), "U_new": torch.empty(U.shape, **f64),
          "costs": torch.empty(batch.k_total, dtype=torch.float32, device=dev),
          "seed": torch.tensor([c["seed"] for c in cases], dtype=torch.int64, device=dev)}
    stream = torch.cuda.current_stream()
    wpg, groups, tune_ms = batch.autotune(io, reps=5, stream=stream)
    one = min(tune_ms[:12])
    eight = min(tune_ms[12:])
    batch.close()
    return {"workload": "batch64[0:8] with K <= 1024: %d sample-steps per tick"
                        % sum(c["cost"]["K"] * c["cost"]["T"] for c in cases),
            "tick_ms_one_lane_per_sample": one, "tick_ms_eight_lanes_per_sample": eight,
            "autotuned": {"waves_per_group": wpg, "groups": groups}}


def graph_update_bench(solver, io, torch, reps=200):
    """The device-resident update replayed from a captured HIP graph: the
    launches of one mppi_update_async (with this io's tick) captured on a
    torch capture stream; the mean from HIP events around all replays, the
    percentiles from events around each."""
    import numpy as np
    gio = dict(io)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        solver.update_async(gio, side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        solver.update_async(gio, torch.cuda.current_stream())
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    for _ in range(20):
        graph.replay()
    mean = span_ms(torch, stream, lambda i: graph.replay(), reps)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for i in range(reps):
        ev[i][0].record(stream)
        graph.replay()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    graph.reset()
    return {"update_ms": mean, "update_hz": 1e3 / mean,
            "update_ms_p5_p50_p95_events_per_replay": [float(np.percentile(ms, x)) for x in (5, 50, 95)]}


def main():
    args = parse()
    if args.cpu_study > 0:
        print(json.dumps({"cpu_study": cpu_study(args.cpu_study)}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2609_02020_amd import binding as B
    from paper_2609_02020_amd import inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    case = inputs.load()[args.workload][args.case]
    K, T, dt = case["cost"]["K"], case["cost"]["T"], case["cost"]["dt"]
    solver = B.Solver(case["robot"], case["cost"], B.FP32)
    dev = torch.device("cuda:0")
    f64 = dict(dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    q = torch.tensor(case["q0"], **f64)
    qd = torch.tensor(case["qd0"], **f64)
    Ua = torch.tensor(case["U_nom"], **f64)
    Ub = torch.empty_like(Ua)
    U_new = torch.empty_like(Ua)
    io = {"q": q, "qd": qd, "target": torch.tensor(B.target_vector(case["target"]), **f64),
          "U_nominal": Ua, "U_new": U_new, "U_shift": Ub,
          "costs": torch.empty(K, dtype=torch.float32, device=dev),
          "status": torch.zeros(1, dtype=torch.int32, device=dev),
          "seed": case["seed"], "tick": 0}

    def update(tick, ev=None):
        io["tick"] = tick
        if ev is not None:
            ev[0].record(stream)
        solver.update_async(io, stream)      # one fused launch: rollouts + Eq. 4
        if ev is not None:
            ev[1].record(stream)
        # warm start: the shifted sequence becomes the next nominal
        io["U_nominal"], io["U_shift"] = io["U_shift"], io["U_nominal"]

    # warm-up: closed loop with the plant (ZOH of u*_0 over dt, 1 ms substeps)
    for w in range(args.warmup):
        update(w)
        solver.plant_step_async(q, qd, U_new[0], dt, max(1, int(round(dt / 1e-3))), stream)
    torch.cuda.synchronize()

    # the timed region: K updates back to back, one pair of HIP events
    # around all of them on the launch stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for s in range(args.steps):
        update(args.warmup + s)
    ev1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    update_ms = ev0.elapsed_time(ev1) / args.steps
    status = int(io["status"].cpu()[0])
    assert status == B.OK, status
    # after it, the spread of single updates, each between its own events
    nd = min(args.steps, 200)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nd)]
    for s in range(nd):
        update(10**6 + s, evs[s])
    torch.cuda.synchronize()
    roll_ms = np.array([a.elapsed_time(b) for a, b in evs])

    ms_per_step = 1e3 * elapsed / args.steps
    rate = args.steps / elapsed
    roll_s = update_ms * 1e-3
    flops = (FLOPS_PER_SAMPLE_STEP * K * T + FLOPS_PER_SAMPLE_TERMINAL * K
             + FLOPS_PER_SAMPLE_ROW_WEIGHT * K * T * 7)
    achieved = flops / roll_s / 1e12

    # host-API rate (PCIe round trip: host state in, U_new and costs out)
    Uh = np.asarray(case["U_nom"], dtype=np.float64)
    qh, qdh = q.cpu().numpy(), qd.cpu().numpy()
    for i in range(10):
        solver.update(qh, qdh, case["target"], Uh, case["seed"], 10**6 + i)
    n_host, th = 200, time.perf_counter()
    host_ms = []
    for i in range(n_host):
        t1 = time.perf_counter()
        st, Uh2, _ = solver.update(qh, qdh, case["target"], Uh, case["seed"], 2 * 10**6 + i)
        host_ms.append(1e3 * (time.perf_counter() - t1))
    host_rate = n_host / (time.perf_counter() - th)

    out = {
        "metric": METRIC, "value": rate, "unit": "Hz", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "%s[%d]: 7-DoF seeded arm, planar wall contact + force cost, "
                               "K=%d, T=%d, dt=%g s" % (args.workload, args.case, K, T, dt),
                   "K": K, "T": T, "dt": dt, "dof": 7, "precision": "fp32 rollouts",
                   "dynamics_route": "composite-rigid-body inertia + LDL^T, eight lanes per sample "
                                     "(default launch); the articulated-body route in aba_rollout_steps_per_s"},
        "rollout_steps_per_s": K * T / roll_s,
        "update_kernel_ms": update_ms,
        "update_kernel_ms_p5_p50_p95_events_per_update": [float(np.percentile(roll_ms, x)) for x in (5, 50, 95)],
        "host_api_update_hz": host_rate,
        "host_api_update_ms_p5_p50_p95": [float(np.percentile(host_ms, x)) for x in (5, 50, 95)],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
                     "traffic": profiled_traffic("update_group_kernel"),
                     "kernel": "update_group_kernel<float, force> + group_merge_kernel (eight lanes per "
                               "sample; the two launches of one update, timed together)",
                     "flops_per_launch": flops,
                     "flops_counted_as": "the method's work per sample-step on the articulated-body route "
                                         "(op-counted per-lane code), credited to the eight-lane route, which "
                                         "computes the same quantities and executes about twice as many"},
    }

    # the same update with the other launch shapes, for comparison
    def shape_ms(waves):
        solver.set_launch(waves)
        for s in range(10):
            update(10**7 + s)
        return span_ms(torch, stream, lambda i: update(10**7 + 10 + i), 100)

    out["launch_shapes"] = {"eight_lanes_per_sample_ms": update_ms,
                            "two_waves_per_64_samples_ms": shape_ms(2),
                            "one_wave_per_64_samples_ms": shape_ms(1)}
    # the articulated-body route (the per-lane kernels): its fastest shape
    aba_ms = min(out["launch_shapes"]["two_waves_per_64_samples_ms"],
                 out["launch_shapes"]["one_wave_per_64_samples_ms"])
    out["aba_rollout_steps_per_s"] = K * T / (aba_ms * 1e-3)
    out["aba_update_hz"] = 1e3 / aba_ms
    solver.set_launch(8)
    out["graph_update"] = graph_update_bench(solver, io, torch)
    # latency-bound at this K: one resident wave per SIMD, T + 1 dependent
    # steps (T rollout steps, then the terminal cost)
    out["roofline"]["waves_resident"] = 4 * ((K + 15) // 16)
    out["roofline"]["per_step_us_upper"] = 1e3 * update_ms / (T + 1)
    if args.batch_ticks > 0:
        out["batch"] = batch_bench(B, inputs.load()["batch64"], torch, dev, args.batch_ticks)
        out["batch_small"] = small_batch_bench(B, inputs.load()["batch64"], torch, dev)
    if not args.no_mlp:
        out["mlp"] = mlp_bench(B, inputs, case["robot"], torch, dev)
    out["collision"] = collision_bench(B, inputs.load()["collision_k4096"][0], torch, dev)
    out["dynamics_routes"] = explicit_bench(B, case, torch, dev)
    out["sampling_variants"] = sampling_bench(B, case, torch, dev)
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = 2 * src.numel() * 4
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_seconds)
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
