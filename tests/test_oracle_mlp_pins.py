"""Pins of the FP64 proposal-network oracle (oracle/mlp.py) against facts
fixed outside it: torch's CPU bfloat16 rounding and tanh-GELU, torch
autograd in FP64 on the same network, central finite differences, and
torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2609_02020_amd import inputs


def torch_net(theta):
    layers = []
    for W, b in mlp.unpack(theta):
        lin = torch.nn.Linear(W.shape[1], W.shape[0], dtype=torch.float64)
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        layers.append(lin)
    return layers


def torch_forward(layers, X):
    a = torch.from_numpy(np.asarray(X, dtype=np.float64))
    for i, lin in enumerate(layers):
        a = lin(a)
        if i < 3:
            a = torch.nn.functional.gelu(a, approximate="tanh")
    return a


def test_layout_and_size():
    assert mlp.N_PARAMS == 169_598
    theta = inputs.draw_mlp_params(1)
    assert theta.shape == (mlp.N_PARAMS,)
    assert np.array_equal(mlp.pack(mlp.unpack(theta)), theta)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(20000) * np.exp2(rng.integers(-40, 40, 20000))).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x.astype(np.float64)), ref)
    # ties go to the even neighbour
    one = 1.0
    assert mlp.bf16(one + 2.0 ** -8) == 1.0
    assert mlp.bf16(one + 3 * 2.0 ** -8) == one + 2.0 ** -6
    assert mlp.bf16(-(one + 3 * 2.0 ** -8)) == -(one + 2.0 ** -6)
    assert mlp.bf16(0.0) == 0.0 and np.isinf(mlp.bf16(np.inf))


def test_gelu_and_derivative():
    z = np.linspace(-8, 8, 4001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="tanh").numpy()
    assert np.abs(mlp.gelu(z) - ref).max() < 1e-14
    zt = torch.from_numpy(z).requires_grad_(True)
    torch.nn.functional.gelu(zt, approximate="tanh").sum().backward()
    assert np.abs(mlp.gelu_prime(z) - zt.grad.numpy()).max() < 1e-13
    h = 1e-5
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.abs(mlp.gelu_prime(z) - fd).max() < 1e-9


def test_exact_network_matches_torch_autograd():
    theta = inputs.draw_mlp_params(5)
    X, Y = inputs.draw_mlp_batch(6, 37)
    layers = torch_net(theta)
    y_t = torch_forward(layers, X)
    y, _ = mlp.forward(theta, X, mirror=False)
    assert np.abs(y - y_t.detach().numpy()).max() < 1e-12
    loss_t = ((y_t - torch.from_numpy(Y)) ** 2).mean()
    loss_t.backward()
    g_t = mlp.pack([(lin.weight.grad.numpy(), lin.bias.grad.numpy()) for lin in layers])
    L, g = mlp.loss_and_grad(theta, X, Y, mirror=False)
    assert L == pytest.approx(loss_t.item(), rel=1e-13)
    assert np.abs(g - g_t).max() <= 1e-12 * np.abs(g_t).max()


def test_exact_gradient_matches_finite_differences():
    theta = inputs.draw_mlp_params(7)
    X, Y = inputs.draw_mlp_batch(8, 9)
    _, g = mlp.loss_and_grad(theta, X, Y, mirror=False)
    rng = np.random.default_rng(9)
    idx = np.concatenate([rng.integers(s.start, s.stop, 6) for w, _, b in mlp.layer_slices()
                          for s in (w, b)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_and_grad(tp, X, Y, mirror=False)[0] - mlp.loss_and_grad(tm, X, Y, mirror=False)[0]) / (2 * h)
        # central difference: O(h^2) truncation plus eps L / h rounding (~1e-11 here)
        assert abs(fd - g[i]) <= 1e-6 * abs(g[i]) + 5e-11, (i, fd, g[i])


def test_mirrored_rounding_stays_within_bf16_error():
    """The BF16-mirrored network differs from the exact one by rounding
    only: outputs within a few bf16 units relative to their scale, and the
    mirrored gradient points the same way as the exact one."""
    theta = inputs.draw_mlp_params(11)
    X, Y = inputs.draw_mlp_batch(12, 64)
    y0, _ = mlp.forward(theta, X, mirror=False)
    y1, _ = mlp.forward(theta, X, mirror=True)
    assert 0 < np.abs(y1 - y0).max() <= 8 * 2.0 ** -8 * np.abs(y0).max()
    _, g0 = mlp.loss_and_grad(theta, X, Y, mirror=False)
    _, g1 = mlp.loss_and_grad(theta, X, Y, mirror=True)
    cos = g0 @ g1 / np.linalg.norm(g0) / np.linalg.norm(g1)
    assert cos > 0.999
    # with every rounding point already exact the two coincide
    thb = mlp.bf16(theta)
    Xb = mlp.bf16(X)
    assert np.array_equal(mlp.bf16(thb), thb) and np.array_equal(mlp.bf16(Xb), Xb)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(13)
    theta = rng.standard_normal(50)
    p = torch.nn.Parameter(torch.from_numpy(theta.copy()))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        p.grad = torch.from_numpy(g.copy())
        opt.step()
        theta, m, v = mlp.adam(theta, m, v, g, t, lr=3e-3)
        assert np.abs(theta - p.detach().numpy()).max() < 1e-14


def test_features_and_torque_scaling(workloads):
    case = workloads["wall_k4096"][0]
    rb, tg = case["robot"], case["target"]
    x = mlp.features(rb, case["q0"], case["qd0"], tg)
    assert x.shape == (21,)
    neg = dict(tg, quat_des=[-c for c in tg["quat_des"]])
    assert np.array_equal(mlp.features(rb, case["q0"], case["qd0"], neg), x)
    assert x[17] >= 0 and abs(np.linalg.norm(x[17:]) - 1) < 1e-15
    U = np.asarray(case["U_nom"])
    assert np.allclose(mlp.torques(rb, mlp.normalised_targets(rb, U)), U, rtol=1e-15, atol=0)
