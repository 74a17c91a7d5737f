"""GPU tests of the proposal network kernels (BF16 matrix cores, FP32
accumulation) against the FP64 oracle with the same BF16 rounding points
(oracle/mlp.py, mirror=True), through the C ABI.

Bars: outputs within 1e-3 of the output scale (max |y|); gradient entries
within 5e-3 of their block's largest oracle entry (per weight matrix and
per bias vector), and each block's error norm within 1e-2 of the oracle
gradient's norm; Adam steps on the GPU's own gradient
within FP32 rounding of the oracle's.  Rows past the batch, padded features
and ragged batch sizes are covered.
"""
import numpy as np
import pytest

from oracle import mlp as om
from paper_2609_02020_amd import binding as B
from paper_2609_02020_amd import inputs
from gpu_util import torch_dev

pytestmark = pytest.mark.gpu
Y_TOL = 1e-3
G_TOL = 1e-2          # relative norm of each block's gradient error
G_ELEM_TOL = 5e-3     # each gradient entry, relative to its block's largest (observed <= 1e-3)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def to_dev(torch, dev, a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float32, device=dev)


def make(workloads, max_batch, seed=1):
    net = B.Mlp(workloads["wall_k4096"][0]["robot"], max_batch)
    theta = f32(inputs.draw_mlp_params(seed))
    net.set_params(theta)
    return net, theta


def check_grad(g_gpu, g_ref, label):
    """Element by element: every entry of each weight matrix and bias
    vector within G_ELEM_TOL of that block's largest oracle entry (a wrong
    tile, lane or padded-edge mapping shows up in single entries); the worst
    entry is printed with its (layer, row, column).  Then the relative norm
    of each block's error as a second bar."""
    for layer, (w, shape, b) in enumerate(om.layer_slices()):
        for sl, name, shp in ((w, "W", shape), (b, "b", (shape[0],))):
            d = np.abs(g_gpu[sl] - g_ref[sl])
            scale = np.abs(g_ref[sl]).max()
            worst = np.unravel_index(int(np.argmax(d)), shp)
            print("%s: layer %d %s worst entry %s |dg| = %.3g of max |g| %.3g (%.2g)"
                  % (label, layer + 1, name, tuple(int(x) for x in worst), d.max(), scale, d.max() / scale))
            assert d.max() <= G_ELEM_TOL * scale, (label, layer + 1, name, worst, d.max() / scale)
            err = np.linalg.norm(g_gpu[sl] - g_ref[sl]) / np.linalg.norm(g_ref[sl])
            assert err <= G_TOL, (label, name, sl, err)


@pytest.mark.parametrize("rows", [1, 63, 64, 200, 512, 2100])
def test_forward_matches_oracle(workloads, rows):
    """2100 rows: 132 workgroups of 16 rows, the last one ragged (4
    rows)."""
    torch, dev = torch_dev()
    net, theta = make(workloads, max(512, rows))
    X, _ = inputs.draw_mlp_batch(rows, rows, scale=1.5)
    X = f32(X)
    y = torch.full((rows, 126), float("nan"), device=dev)
    net.forward_async(to_dev(torch, dev, X), y)
    torch.cuda.synchronize()
    y_ref, _ = om.forward(theta, X, mirror=True)
    err = np.abs(y.cpu().numpy() - y_ref).max() / np.abs(y_ref).max()
    print("rows %d: max |dy| / max |y| = %.3g" % (rows, err))
    assert err <= Y_TOL
    net.close()


@pytest.mark.parametrize("rows", [37, 256, 300, 2000, 2100])
def test_gradient_matches_oracle(workloads, rows):
    """2000 rows: 16 k-steps of 32 rows per weight-gradient wave (four load
    chunks) for the weight and bias gradients; 2100 rows: a batch that is
    not a multiple of 64 (padding rows in the last forward workgroups and
    the last k-step)."""
    torch, dev = torch_dev()
    net, theta = make(workloads, max(512, rows), seed=2)
    X, Y = inputs.draw_mlp_batch(100 + rows, rows)
    X, Y = f32(X), f32(Y)
    g = torch.full((B.MLP_PARAMS,), float("nan"), device=dev)
    loss = torch.full((1,), float("nan"), device=dev)
    net.grad_async(to_dev(torch, dev, X), to_dev(torch, dev, Y), g, loss)
    torch.cuda.synchronize()
    L_ref, g_ref = om.loss_and_grad(theta, X, Y, mirror=True)
    g_gpu = g.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - L_ref) <= 1e-3 * L_ref
    check_grad(g_gpu, g_ref, "rows %d" % rows)
    # and the exact FP64 gradient of the unrounded network points the same way
    _, g_exact = om.loss_and_grad(theta, X, Y, mirror=False)
    assert g_gpu @ g_exact / np.linalg.norm(g_gpu) / np.linalg.norm(g_exact) > 0.999
    net.close()


def test_forward_rows_independent_of_batch(workloads):
    """Rows never mix in the forward pass, so the first 500 rows of a
    2100-row batch get the bits that a 500-row batch gives them."""
    torch, dev = torch_dev()
    net, _ = make(workloads, 2100, seed=4)
    X, Y = inputs.draw_mlp_batch(77, 2100)
    Xd = to_dev(torch, dev, X)
    y_big = torch.zeros((2100, 126), device=dev)
    y_small = torch.zeros((500, 126), device=dev)
    net.forward_async(Xd, y_big)
    net.forward_async(Xd[:500].contiguous(), y_small)
    torch.cuda.synchronize()
    assert torch.equal(y_big[:500], y_small)
    net.close()


def test_smaller_batch_after_larger_ignores_stale_rows(workloads):
    """A batch of 70 rows after one of 512: the weight gradients contract
    only the rows of the current batch."""
    torch, dev = torch_dev()
    net, theta = make(workloads, 512, seed=3)
    X1, Y1 = inputs.draw_mlp_batch(31, 512)
    net.grad_async(to_dev(torch, dev, f32(X1)), to_dev(torch, dev, f32(Y1)))
    X, Y = inputs.draw_mlp_batch(32, 70)
    X, Y = f32(X), f32(Y)
    g = torch.zeros(B.MLP_PARAMS, device=dev)
    net.grad_async(to_dev(torch, dev, X), to_dev(torch, dev, Y), g)
    torch.cuda.synchronize()
    _, g_ref = om.loss_and_grad(theta, X, Y, mirror=True)
    check_grad(g.cpu().numpy().astype(np.float64), g_ref, "70 after 512")
    net.close()


def test_adam_steps_match_oracle(workloads):
    torch, dev = torch_dev()
    net, theta = make(workloads, 256, seed=4)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for t in (1, 2, 3):
        X, Y = inputs.draw_mlp_batch(40 + t, 128)
        g = torch.zeros(B.MLP_PARAMS, device=dev)
        net.grad_async(to_dev(torch, dev, f32(X)), to_dev(torch, dev, f32(Y)), g)
        net.adam_async(lr=2e-3)
        torch.cuda.synchronize()
        theta, m, v = om.adam(theta, m, v, g.cpu().numpy().astype(np.float64), t, lr=2e-3)
        got = net.get_params().astype(np.float64)
        # FP32 master weights: a few units of FP32 rounding of |theta| + lr
        assert np.abs(got - theta).max() <= 4e-7 * (np.abs(theta).max() + 2e-3), t
        theta = got   # continue from the GPU's FP32 state
    net.close()


@pytest.mark.parametrize("rows", [128, 2000])
def test_train_step_equals_grad_then_adam(workloads, rows):
    """The one-call training step (Adam applied inside the weight-gradient
    launch as each tile completes) leaves the same master weights, BF16
    copies, loss and step count as separate gradient and Adam calls: bit
    for bit over three steps, and the next forward agrees bit for bit."""
    torch, dev = torch_dev()
    a, _ = make(workloads, rows, seed=8)
    b, _ = make(workloads, rows, seed=8)
    la = torch.zeros(1, device=dev)
    lb = torch.zeros(1, device=dev)
    for t in range(3):
        X, Y = inputs.draw_mlp_batch(60 + t, rows)
        Xd, Yd = to_dev(torch, dev, f32(X)), to_dev(torch, dev, f32(Y))
        a.train_step_async(Xd, Yd, la, lr=2e-3)
        b.grad_async(Xd, Yd, loss=lb)
        b.adam_async(lr=2e-3)
        torch.cuda.synchronize()
        assert la.item() == lb.item(), t
        assert np.array_equal(a.get_params(), b.get_params()), t
    X, _ = inputs.draw_mlp_batch(70, rows)
    ya = torch.zeros((rows, 126), device=dev)
    yb = torch.zeros((rows, 126), device=dev)
    a.forward_async(to_dev(torch, dev, f32(X)), ya)
    b.forward_async(to_dev(torch, dev, f32(X)), yb)
    torch.cuda.synchronize()
    assert torch.equal(ya, yb)
    a.close()
    b.close()


def test_network_entry_points_reject_bad_sizes_and_adam_parameters(workloads):
    """Batches beyond the network's capacity and invalid Adam parameters are
    refused on the host before any launch; a refused training step leaves
    the parameters and the Adam step count unchanged."""
    torch, dev = torch_dev()
    net, theta = make(workloads, 64, seed=9)
    x = torch.zeros((65, 21), device=dev)
    y = torch.zeros((65, 126), device=dev)
    with pytest.raises(B.MppiError):
        net.grad_async(x, y)
    with pytest.raises(B.MppiError):
        net.train_step_async(x, y)
    with pytest.raises(B.MppiError):
        net.forward_async(x, torch.zeros((65, 126), device=dev))
    q = torch.zeros((65, 7), dtype=torch.float64, device=dev)
    tg = torch.zeros((65, 13), dtype=torch.float64, device=dev)
    tg[:, 3] = 1.0
    with pytest.raises(B.MppiError):
        net.propose_async(q, q, tg, torch.zeros((65, 126), dtype=torch.float64, device=dev))
    x64, y64 = x[:64].contiguous(), y[:64].contiguous()
    for bad in (dict(lr=-1.0), dict(beta1=1.0), dict(beta2=-0.1), dict(eps=0.0)):
        with pytest.raises(B.MppiError):
            net.train_step_async(x64, y64, **bad)
        with pytest.raises(B.MppiError):
            net.adam_async(**bad)
    torch.cuda.synchronize()
    assert np.array_equal(net.get_params(), theta)
    # the first accepted step is Adam step 1 (bias corrections of t = 1)
    X, Y = inputs.draw_mlp_batch(80, 64)
    g = torch.zeros(B.MLP_PARAMS, device=dev)
    net.grad_async(to_dev(torch, dev, f32(X)), to_dev(torch, dev, f32(Y)), g)
    net.adam_async(lr=2e-3)
    torch.cuda.synchronize()
    ref, _, _ = om.adam(theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size),
                        g.cpu().numpy().astype(np.float64), 1, lr=2e-3)
    got = net.get_params().astype(np.float64)
    assert np.abs(got - ref).max() <= 4e-7 * (np.abs(ref).max() + 2e-3)
    net.close()


def test_training_reduces_loss_and_keeps_weight_copies_consistent(workloads):
    """300 Adam steps on a smooth synthetic regression; afterwards the GPU
    forward and gradient (which read the BF16 copies and their transposes
    written by the Adam kernel) still match the oracle on the trained
    master weights."""
    torch, dev = torch_dev()
    net, _ = make(workloads, 256, seed=5)
    rng = np.random.default_rng(6)
    A = rng.standard_normal((21, 126)) / np.sqrt(21)
    Xall = rng.uniform(-1, 1, size=(4096, 21))
    Yall = 0.5 * np.tanh(Xall @ A)
    Xd, Yd = to_dev(torch, dev, f32(Xall)), to_dev(torch, dev, f32(Yall))
    loss = torch.zeros(1, device=dev)
    hist = []
    for step in range(300):
        i = (step * 256) % 4096
        net.train_step_async(Xd[i:i + 256], Yd[i:i + 256], loss, lr=1e-3)
        if step % 50 == 0 or step == 299:
            torch.cuda.synchronize()
            hist.append(loss.item())
    print("loss:", np.round(hist, 5))
    assert hist[-1] < 0.2 * hist[0]
    theta = net.get_params().astype(np.float64)
    X, Y = f32(Xall[:200]), f32(Yall[:200])
    y = torch.zeros((200, 126), device=dev)
    net.forward_async(to_dev(torch, dev, X), y)
    g = torch.zeros(B.MLP_PARAMS, device=dev)
    net.grad_async(to_dev(torch, dev, X), to_dev(torch, dev, Y), g)
    torch.cuda.synchronize()
    y_ref, _ = om.forward(theta, X, mirror=True)
    assert np.abs(y.cpu().numpy() - y_ref).max() <= Y_TOL * np.abs(y_ref).max()
    _, g_ref = om.loss_and_grad(theta, X, Y, mirror=True)
    check_grad(g.cpu().numpy().astype(np.float64), g_ref, "after training")
    net.close()


def test_propose_matches_oracle(workloads):
    """Features from device states and targets, forward, torque scaling."""
    torch, dev = torch_dev()
    cases = workloads["wall_k4096"][:5]
    rb = cases[0]["robot"]
    net = B.Mlp(rb, 64)
    theta = f32(inputs.draw_mlp_params(7))
    net.set_params(theta)
    rng = np.random.default_rng(8)
    q = np.array([c["q0"] for c in cases]) + rng.uniform(-0.3, 0.3, (5, 7))
    qd = rng.uniform(-1, 1, (5, 7))
    tg = np.array([B.target_vector(c["target"]) for c in cases])
    tg[1, 3:7] *= -2.0   # unnormalised, w < 0
    U = torch.full((5, 130), float("nan"), dtype=torch.float64, device=dev)
    net.propose_async(to_dev(torch, dev, q, torch.float64), to_dev(torch, dev, qd, torch.float64),
                      to_dev(torch, dev, tg, torch.float64), U, u_stride=130)
    torch.cuda.synchronize()
    Ug = U.cpu().numpy()
    assert np.isnan(Ug[:, 126:]).all()
    for p, c in enumerate(cases):
        t = {"p_des": tg[p, :3], "quat_des": tg[p, 3:7]}
        x = f32(om.features(rb, q[p], qd[p], t))
        y, _ = om.forward(theta, x[None], mirror=True)
        U_ref = om.torques(rb, y[0])
        tau = om.torque_scale(rb)
        assert np.abs(Ug[p, :126].reshape(18, 7) - U_ref).max() <= Y_TOL * np.abs(y).max() * tau.max()
    net.close()


@pytest.mark.parametrize("n", [1, 16, 17, 64])
def test_propose_equals_forward_of_encoded_rows(workloads, n):
    """The proposal (features encoded inside its one forward launch) and the
    two-step path (encode the rows, forward them, scale by tau_max) give the
    same torques bit for bit, over whole and ragged workgroups of 16 rows."""
    torch, dev = torch_dev()
    cases = workloads["wall_k4096"][:4]
    rb = cases[0]["robot"]
    net = B.Mlp(rb, 64)
    net.set_params(f32(inputs.draw_mlp_params(9)))
    rng = np.random.default_rng(20 + n)
    q = to_dev(torch, dev, rng.uniform(-2, 2, (n, 7)), torch.float64)
    qd = to_dev(torch, dev, rng.uniform(-2, 2, (n, 7)), torch.float64)
    tg = np.array([B.target_vector(cases[i % 4]["target"]) for i in range(n)])
    tg[::3, 3:7] *= -1.5   # unnormalised, w < 0
    tg = to_dev(torch, dev, tg, torch.float64)
    U = torch.full((n, 126), float("nan"), dtype=torch.float64, device=dev)
    net.propose_async(q, qd, tg, U)
    x = torch.zeros((n, 21), dtype=torch.float32, device=dev)
    y = torch.zeros((n, 126), dtype=torch.float32, device=dev)
    net.encode_async(q, qd, tg, x)
    net.forward_async(x, y)
    torch.cuda.synchronize()
    expect = y.cpu().numpy().astype(np.float64) * np.tile(om.torque_scale(rb), 18)
    assert np.array_equal(U.cpu().numpy(), expect)
    net.close()


def test_select_nominal_keeps_the_cheaper_sequence(ora, workloads):
    """Noise-free rollout costs of the warm start and of a candidate against
    the oracle's rollout with sigma = 0; the candidate replaces the nominal
    only when it is cheaper (both directions exercised)."""
    torch, dev = torch_dev()
    f64 = dict(dtype=torch.float64, device=dev)
    for i, case in enumerate(workloads["wall_k4096"][:3]):
        cost = case["cost"]
        solver = B.Solver(case["robot"], cost, B.FP32)
        U0 = np.asarray(case["U_nom"])
        rng = np.random.default_rng(20 + i)
        for cand in (U0 + rng.normal(size=U0.shape) * 4.0, U0 + rng.normal(size=U0.shape) * 0.05):
            c0 = ora.rollout(case["robot"], dict(cost, sigma=[0.0] * 7), case["target"], case["q0"],
                             case["qd0"], U0, 0, 0, 0)[0]
            c1 = ora.rollout(case["robot"], dict(cost, sigma=[0.0] * 7), case["target"], case["q0"],
                             case["qd0"], cand, 0, 0, 0)[0]
            io = {"q": torch.tensor(case["q0"], **f64), "qd": torch.tensor(case["qd0"], **f64),
                  "target": torch.tensor(B.target_vector(case["target"]), **f64),
                  "U_nominal": torch.tensor(U0, **f64), "seed": 0, "tick": 0}
            costs = torch.zeros(2, **f64)
            solver.select_nominal_async(io, torch.tensor(cand, **f64), costs)
            torch.cuda.synchronize()
            cg = costs.cpu().numpy()
            assert abs(cg[0] - c0) <= 1e-4 * abs(c0) and abs(cg[1] - c1) <= 1e-4 * abs(c1), (cg, c0, c1)
            if abs(c1 - c0) > 1e-3 * abs(c0):
                expect = cand if c1 < c0 else U0
                assert np.array_equal(io["U_nominal"].cpu().numpy(), expect)
        solver.close()


def test_batch_plant_and_select_match_single_problem(workloads):
    torch, dev = torch_dev()
    f64 = dict(dtype=torch.float64, device=dev)
    cases = []
    for i, c in enumerate(workloads["batch64"][:6]):
        T = c["cost"]["T"]
        cases.append(dict(c, cost=dict(c["cost"], K=256 + 64 * i), U_nom=np.asarray(c["U_nom"])[:T]))
    batch = B.Batch([(c["robot"], c["cost"]) for c in cases])
    U = np.zeros((batch.u_total // 7, 7))
    rng = np.random.default_rng(9)
    Uc = np.zeros_like(U)
    for p, c in enumerate(cases):
        sl = slice(batch.u_off[p] // 7, batch.u_off[p] // 7 + batch.T[p])
        U[sl] = c["U_nom"]
        Uc[sl] = c["U_nom"] + rng.normal(size=c["U_nom"].shape) * (0.05 if p % 2 else 3.0)
    io = {"q": torch.tensor(np.array([c["q0"] for c in cases]), **f64),
          "qd": torch.tensor(np.array([c["qd0"] for c in cases]), **f64),
          "target": torch.tensor(np.array([B.target_vector(c["target"]) for c in cases]), **f64),
          "U_nominal": torch.tensor(U, **f64), "U_new": torch.tensor(Uc, **f64),
          "seed": torch.arange(len(cases), dtype=torch.int64, device=dev)}
    costs = torch.zeros((len(cases), 2), **f64)
    batch.select_nominal_async(io, torch.tensor(Uc, **f64), costs)
    batch.plant_step_async(io, 0.01, 10)
    torch.cuda.synchronize()
    for p, c in enumerate(cases):
        sl = slice(batch.u_off[p] // 7, batch.u_off[p] // 7 + batch.T[p])
        solver = B.Solver(c["robot"], c["cost"], B.FP32)
        io1 = {"q": torch.tensor(c["q0"], **f64), "qd": torch.tensor(c["qd0"], **f64),
               "target": torch.tensor(B.target_vector(c["target"]), **f64),
               "U_nominal": torch.tensor(U[sl], **f64), "seed": 0, "tick": 0}
        c1 = torch.zeros(2, **f64)
        solver.select_nominal_async(io1, torch.tensor(Uc[sl], **f64), c1)
        q1 = torch.tensor(c["q0"], **f64)
        qd1 = torch.tensor(c["qd0"], **f64)
        solver.plant_step_async(q1, qd1, torch.tensor(Uc[sl][0], **f64), 0.01, 10)
        torch.cuda.synchronize()
        assert np.allclose(costs[p].cpu().numpy(), c1.cpu().numpy(), rtol=1e-5, atol=0), p
        assert np.array_equal(io["U_nominal"][sl].cpu().numpy(), io1["U_nominal"].cpu().numpy()), p
        # the same FP64 plant code in two kernels (contraction may differ)
        assert np.abs(io["q"][p].cpu().numpy() - q1.cpu().numpy()).max() <= 1e-12, p
        assert np.abs(io["qd"][p].cpu().numpy() - qd1.cpu().numpy()).max() <= 1e-10, p
        solver.close()
    batch.close()


def test_encode_rows_match_oracle(workloads):
    """Training rows: features and torque-limit-normalised targets."""
    torch, dev = torch_dev()
    cases = workloads["wall_k4096"][:4]
    rb = cases[0]["robot"]
    net = B.Mlp(rb, 64)
    rng = np.random.default_rng(12)
    n = 300   # more rows than the network's batch capacity
    q = rng.uniform(-2, 2, (n, 7))
    qd = rng.uniform(-2, 2, (n, 7))
    tg = np.array([B.target_vector(cases[i % 4]["target"]) for i in range(n)])
    U = rng.uniform(-80, 80, (n, 126))
    x = torch.zeros((n, 21), device=dev)
    y = torch.zeros((n, 126), device=dev)
    net.encode_async(to_dev(torch, dev, q, torch.float64), to_dev(torch, dev, qd, torch.float64),
                     to_dev(torch, dev, tg, torch.float64), x, U=to_dev(torch, dev, U, torch.float64), y=y)
    torch.cuda.synchronize()
    for p in range(n):
        t = {"p_des": tg[p, :3], "quat_des": tg[p, 3:7]}
        assert np.abs(x[p].cpu().numpy() - om.features(rb, q[p], qd[p], t)).max() <= 1e-6
        assert np.abs(y[p].cpu().numpy() - om.normalised_targets(rb, U[p].reshape(18, 7))).max() <= 1e-6
    net.close()
