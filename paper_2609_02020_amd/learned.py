"""Learned proposal: closed-loop data from plain MPPI, training on the GPU,
and closed-loop runs with the proposal as a candidate nominal sequence.

Everything here orchestrates library calls (binding.Batch, binding.Mlp);
the rollouts, the plant, the selection, the network's forward and backward
passes and Adam all run in the library's kernels.  torch only holds device
memory.

A closed loop runs many episodes of one task as one batch: per control tick
(dt, Philox tick = tick index) it optionally asks the proposal for a mean
sequence and keeps it as the nominal only where its noise-free rollout is
cheaper than the shifted warm start (plain MPPI stays the fallback), runs
one batched update, applies the first row of U_new to the FP64 plant for
dt (1 ms substeps) and shifts U_new into the next warm start.
"""
from __future__ import annotations

import math

import numpy as np

from . import binding as B


def _device(torch):
    assert torch.cuda.is_available(), "the learned-proposal path needs a GPU"
    return torch.device("cuda:0")


def closed_loop(robot, cost, episodes, K, ticks, proposal=None, stream=None, record_U=False):
    """Runs len(episodes) episodes for `ticks` ticks at K samples.  Returns
    device tensors: q, qd [ticks][n][7] (state at each tick, before the
    update), u [ticks][n][7] (applied torque: first row of U_new), target
    [n][13], U [ticks][n][18*7] (U_new) when record_U, and picked
    [ticks][n] (1 where the proposal was taken)."""
    import torch
    dev = _device(torch)
    n, T = len(episodes), int(cost["T"])
    c = dict(cost, K=int(K))
    batch = B.Batch([(robot, c)] * n)
    assert batch.u_off == [p * T * 7 for p in range(n)]
    f64 = dict(dtype=torch.float64, device=dev)
    U0 = np.array([np.asarray(e["U_nom"], dtype=np.float64)[:T] for e in episodes]).reshape(n * T, 7)
    io = {"q": torch.tensor(np.array([e["q0"] for e in episodes]), **f64),
          "qd": torch.tensor(np.array([e["qd0"] for e in episodes]), **f64),
          "target": torch.tensor(np.array([B.target_vector(e["target"]) for e in episodes]), **f64),
          "U_nominal": torch.tensor(U0, **f64), "U_new": torch.empty((n * T, 7), **f64),
          "U_shift": torch.empty((n * T, 7), **f64),
          "status": torch.zeros(n, dtype=torch.int32, device=dev),
          "seed": torch.tensor([int(e["seed"]) for e in episodes], dtype=torch.int64, device=dev)}
    out = {"q": torch.empty((ticks, n, 7), **f64), "qd": torch.empty((ticks, n, 7), **f64),
           "u": torch.empty((ticks, n, 7), **f64), "target": io["target"],
           "picked": torch.zeros((ticks, n), dtype=torch.int32, device=dev)}
    if record_U:
        out["U"] = torch.empty((ticks, n, T * 7), **f64)
    cand = torch.empty((n * T, 7), **f64) if proposal is not None else None
    sel = torch.empty((n, 2), **f64) if proposal is not None else None
    dt = float(cost["dt"])
    sub = max(1, int(round(dt / 1e-3)))
    for t in range(ticks):
        out["q"][t].copy_(io["q"])
        out["qd"][t].copy_(io["qd"])
        if proposal is not None:
            proposal.propose_async(io["q"], io["qd"], io["target"], cand, u_stride=T * 7, stream=stream)
            batch.select_nominal_async(io, cand, sel, stream=stream)
            out["picked"][t].copy_((sel[:, 1] < sel[:, 0]).to(torch.int32))
        batch.update_async(io, tick=t, stream=stream)
        Unew = io["U_new"].view(n, T * 7)
        out["u"][t].copy_(Unew[:, :7])
        if record_U:
            out["U"][t].copy_(Unew)
        batch.plant_step_async(io, dt, sub, stream=stream)
        io["U_nominal"], io["U_shift"] = io["U_shift"], io["U_nominal"]
    torch.cuda.synchronize()
    st = io["status"].cpu().numpy()
    batch.close()
    out["status"] = st
    return out


def make_dataset(robot, cost, episodes, K=4096, ticks=200, group=64, stream=None, log=None):
    """(state, target) -> U* pairs from plain-MPPI closed loops at K samples:
    one row per episode and tick.  Returns device tensors q, qd [N][7],
    target [N][13], U [N][126]."""
    import torch
    parts = {"q": [], "qd": [], "target": [], "U": []}
    for g0 in range(0, len(episodes), group):
        eps = episodes[g0:g0 + group]
        r = closed_loop(robot, cost, eps, K, ticks, stream=stream, record_U=True)
        n = len(eps)
        parts["q"].append(r["q"].reshape(ticks * n, 7))
        parts["qd"].append(r["qd"].reshape(ticks * n, 7))
        parts["target"].append(r["target"].unsqueeze(0).expand(ticks, n, 13).reshape(ticks * n, 13))
        parts["U"].append(r["U"].reshape(ticks * n, -1))
        if log:
            log("dataset: episodes %d-%d done" % (g0, g0 + n - 1))
    return {k: torch.cat(v).contiguous() for k, v in parts.items()}


def train(net, data, epochs=30, batch=512, lr=1e-3, seed=0, stream=None, log=None):
    """Adam on the MSE of the torque-limit-normalised sequences; the rows are
    encoded once (mppi_mlp_encode_async) and visited in a seeded order per
    epoch; cosine learning-rate decay.  Returns the loss of the initial
    parameters (first 16 batches) followed by the mean loss of every epoch."""
    import torch
    dev = _device(torch)
    N = data["q"].shape[0]
    X = torch.empty((N, B.MLP_INPUTS), dtype=torch.float32, device=dev)
    Y = torch.empty((N, B.MLP_OUTPUTS), dtype=torch.float32, device=dev)
    net.encode_async(data["q"], data["qd"], data["target"], X, U=data["U"], y=Y, u_stride=data["U"].shape[1],
                     stream=stream)
    rng = np.random.default_rng(seed)
    steps = N // batch
    losses = torch.zeros(steps, dtype=torch.float32, device=dev)
    # loss of the initial parameters on the first rows (no update)
    for s in range(min(steps, 16)):
        net.grad_async(X[s * batch:(s + 1) * batch], Y[s * batch:(s + 1) * batch], loss=losses[s:s + 1],
                       stream=stream)
    torch.cuda.synchronize()
    hist = [float(losses[:min(steps, 16)].mean().item())]
    if log:
        log("initial loss %.5f" % hist[0])
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).to(dev)
        Xs, Ys = X.index_select(0, perm), Y.index_select(0, perm)
        lr_e = lr * 0.5 * (1.0 + math.cos(math.pi * ep / epochs))
        for s in range(steps):
            net.train_step_async(Xs[s * batch:(s + 1) * batch], Ys[s * batch:(s + 1) * batch], losses[s:s + 1],
                                 lr=lr_e, stream=stream)
        torch.cuda.synchronize()
        hist.append(float(losses.mean().item()))
        if log:
            log("epoch %d: lr %.2e, loss %.5f" % (ep, lr_e, hist[-1]))
    return hist
