"""Helpers for the GPU tests: device buffers for one update and the parity
criteria (per-sample cost relative error, U_new absolute error in N m)."""
import numpy as np

from paper_2609_02020_amd import binding as B

COST_RTOL = 1e-4      # per-sample cost, relative to the FP64 oracle
U_ATOL = 1e-3         # U_new, N m
U32 = 2.0 ** -24      # FP32 unit roundoff
KAPPA_CAP = 1e-2      # the largest per-sample cost error allowed anywhere (FP32)


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    return torch, torch.device("cuda:0")


def device_update(solver, case, seed, tick, precision=B.FP32, stage=False, costs_in=None,
                  noise_in=None, U_nom=None):
    """Runs one device-side update; returns numpy copies of U_new, U_shift,
    costs, noise [K, T, 7] and the status word."""
    torch, dev = torch_dev()
    K, T = solver.K, solver.T
    rdt = torch.float64 if precision == B.FP64 else torch.float32
    f64 = dict(dtype=torch.float64, device=dev)
    U = np.asarray(case["U_nom"] if U_nom is None else U_nom, dtype=np.float64)
    io = {
        "q": torch.tensor(case["q0"], **f64),
        "qd": torch.tensor(case["qd0"], **f64),
        "target": torch.tensor(B.target_vector(case["target"]), **f64),
        "U_nominal": torch.tensor(U, **f64).contiguous(),
        "U_new": torch.full((T, 7), float("nan"), **f64),
        "U_shift": torch.full((T, 7), float("nan"), **f64),
        "costs": costs_in if costs_in is not None else torch.full((K,), float("nan"), dtype=rdt, device=dev),
        "noise": noise_in if noise_in is not None else torch.full((T * 7 * K,), float("nan"), dtype=rdt, device=dev),
        "status": torch.full((1,), -1, dtype=torch.int32, device=dev),
        "seed": seed, "tick": tick,
    }
    if stage:
        solver.weights_async(io)
    else:
        solver.update_async(io)
    torch.cuda.synchronize()
    noise = io["noise"].double().cpu().numpy().reshape(T, 7, K).transpose(2, 0, 1).copy()
    return {"U_new": io["U_new"].cpu().numpy(), "U_shift": io["U_shift"].cpu().numpy(),
            "costs": io["costs"].double().cpu().numpy(), "noise": noise,
            "status": int(io["status"].cpu().numpy()[0]), "io": io}


def check_noise_fp32(E_gpu, E_ref, sigma, label=""):
    """FP32 perturbations [K, T, 7] of i.i.d. sampling against the oracle's
    FP64 ones from the same Philox bits, element by element.  The kernels
    form the radius uniform u = (x + 1) 2^-32 in FP32, which near u = 1 is
    resolved to 2^-24 only, so the Box-Muller radius r = sqrt(-2 ln u)
    carries an absolute error of about 2^-24 / r (at most sqrt(2^-23),
    when u rounds to 1); with |z| <= r that is at most 2^-24 / |z|.  A
    normal z of the oracle may therefore differ by min(2^-22 / |z|, 4e-4)
    (twice the estimate) plus 2e-5 for the rest of the FP32 arithmetic
    (hardware log2, sin and cos), scaled by sigma_j."""
    sig = np.asarray(sigma, dtype=float)[:E_ref.shape[-1]]
    z = np.abs(E_ref) / np.where(sig > 0, sig, 1.0)
    tol = 2e-5 + sig * np.minimum(2.0 ** -22 / np.maximum(z, 1e-30), 4e-4)
    diff = np.abs(E_gpu - E_ref)
    i = np.unravel_index(int(np.argmax(diff / tol)), diff.shape)
    print("%s: noise max |d| %.3g; tightest element |d| %.3g at |du| %.3g (bound %.3g)"
          % (label, diff.max(), diff[i], abs(E_ref[i]), tol[i]))
    assert diff[i] <= tol[i], (label, diff[i], tol[i])


def cost_rel_err(S_gpu, S_ref):
    return np.abs(S_gpu - S_ref) / np.maximum(np.abs(S_ref), 1e-9)


def check_update(ora, case, out, lam, S_ref, U_ref, label=""):
    """The two parity criteria for U_new: (1) stage-isolated: the oracle's
    Eq. 4 weighting of the GPU's own costs and noise reproduces the GPU
    U_new; (2) end-to-end against the full oracle update whenever the cost
    errors cannot move the weights (max |dS| / lambda <= 1e-3).  Returns a
    note when (2) is not applicable (a precision finding, not a failure)."""
    st, U_stage, _ = ora.weights_update(out["costs"], out["noise"], case["U_nom"], lam)
    assert st == 0
    assert np.abs(out["U_new"] - U_stage).max() <= U_ATOL, label
    dS = np.abs(out["costs"] - S_ref).max() / lam
    if dS <= 1e-3:
        assert np.abs(out["U_new"] - U_ref).max() <= U_ATOL, label
        return None
    order = np.argsort(S_ref)
    return "%s: max|dS|/lambda = %.3g > 1e-3 (top-2 gap %.3g); end-to-end |dU| = %.3g N m" % (
        label, dS, S_ref[order[1]] - S_ref[order[0]], np.abs(out["U_new"] - U_ref).max())


def force_condition(ora, case, seed, tick, k):
    """Largest condition number of J M^-1 J^T (the inverse operational-space
    inertia inverted by the force estimate of Eq. 13) over the pre-step
    states of the oracle trajectory of sample k."""
    rb, cost = case["robot"], case["cost"]
    q, qd = np.array(case["q0"], float), np.array(case["qd0"], float)
    U = np.asarray(case["U_nom"], float)
    _, E = ora.rollout(rb, cost, case["target"], case["q0"], case["qd0"], U, seed, tick, k)
    worst = 1.0
    for t in range(cost["T"]):
        v = U[t] + E[t]
        J = ora.ee_jacobian(rb, q)
        M = ora.mass_jacobian_sum(rb, q)
        worst = max(worst, np.linalg.cond(J @ np.linalg.solve(M, J.T)))
        f = None
        if cost.get("ext_mode", 0) == 2:
            _, _, pe, _ = ora.fk(rb, q)
            f = np.concatenate([ora.wall_force(cost, pe, J[:3] @ qd), np.zeros(3)])
        qd = qd + ora.aba(rb, q, qd, v, f) * cost["dt"]
        q = q + qd * cost["dt"]
    return worst


def check_costs_fp32(ora, case, S_gpu, S_ref, seed, tick, label=""):
    """Per-sample cost parity for FP32 rollouts: relative error <= 1e-4, or,
    for a sample whose force estimate inverts an ill-conditioned matrix
    (condition number kappa of J M^-1 J^T along its trajectory), <=
    min(kappa * u32, KAPPA_CAP): kappa u32 is the forward-error scale of a
    backward-stable FP32 solve of that matrix (the least-squares solve the
    kernels use stays well inside it), and no sample may be further than
    KAPPA_CAP from the oracle however ill-conditioned.  Prints and returns
    every such sample (k, error, kappa)."""
    err = cost_rel_err(S_gpu, S_ref)
    flagged = []
    has_force = any(w != 0 for w in case["cost"]["W_force"]) or any(w != 0 for w in case["cost"]["W_reg"])
    for k in np.nonzero(err > COST_RTOL)[0]:
        assert has_force, "%s: sample %d rel err %.3g without the force term" % (label, k, err[k])
        kappa = force_condition(ora, case, seed, tick, int(k))
        bound = min(kappa * U32, KAPPA_CAP)
        print("%s: flagged sample k=%d rel err %.3g kappa %.3g bound %.3g" % (label, k, err[k], kappa, bound))
        assert err[k] <= bound, "%s: sample %d rel err %.3g, kappa %.3g" % (label, k, err[k], kappa)
        flagged.append((int(k), float(err[k]), float(kappa)))
    return flagged
