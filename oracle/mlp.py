"""FP64 CPU oracle of the learned proposal network (TEST INFRASTRUCTURE ONLY).

Only ``tests/`` import this module; the product library never does, and it
shares no code with the HIP kernels.

The proposal is an addition to the method of the paper (which samples around
the shifted warm start only): a multilayer perceptron maps the measured state
and the pose target to a mean torque sequence over the horizon, which is then
offered as an alternative nominal sequence for the sampling of Eq. 2.  Plain
numpy, one line per formula:

  features   x = (q / q_max, qd / qd_max, p_des, quat_des) in R^21, the
             quaternion (w, x, y, z) normalised and sign-fixed to w >= 0
  network    z_l = W_l a_{l-1} + b_l,  a_l = gelu(z_l)  (l = 1, 2, 3),
             y = W_4 a_3 + b_4 in R^126, widths 21-256-256-256-126
  output     U[t, j] = tau_max_j * y[7 t + j]   (T = 18 steps, 7 joints)
  loss       L = sum (y - y*)^2 / (B * 126) over a batch of B rows, with
             y*[7 t + j] = U*[t, j] / tau_max_j
  gelu       the tanh form of Hendrycks and Gimpel (2016):
             gelu(z) = z/2 (1 + tanh(c (z + 0.044715 z^3))), c = sqrt(2/pi)
  Adam       Kingma and Ba (2015), Algorithm 1, bias-corrected moments.

``mirror=True`` reproduces the rounding points of the BF16 kernels: the
weights, the input features, the hidden activations a_l and the backward
signals e_l = dL/dz_l are rounded to bfloat16 (round to nearest, ties to
even, 8 significant bits) where the kernels store them; everything else is
FP64 here (FP32 in the kernels).  The backward pass then differentiates
through the rounding as the identity, as the kernels do.  ``mirror=False``
is the exact FP64 network and its exact gradient.

Flat parameter layout (shared by the C ABI): for l = 1..4, W_l row-major
[out][in], then b_l [out]; 169,598 values.
"""
from __future__ import annotations

import numpy as np

DIMS = (21, 256, 256, 256, 126)
T_STEPS, NJ = 18, 7
GELU_C = np.sqrt(2.0 / np.pi)
GELU_A = 0.044715


def layer_slices():
    """[(W slice, W shape, b slice)] for the four layers of the flat vector."""
    out, o = [], 0
    for i in range(4):
        n_in, n_out = DIMS[i], DIMS[i + 1]
        w = slice(o, o + n_out * n_in)
        o += n_out * n_in
        b = slice(o, o + n_out)
        o += n_out
        out.append((w, (n_out, n_in), b))
    return out


N_PARAMS = layer_slices()[-1][2].stop


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits, ties to even,
    FP32 exponent range), returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                      # x = m 2^e, 0.5 <= |m| < 1
    r = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    return np.where(np.isfinite(x), r, x)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_A * z ** 3)))


def gelu_prime(z):
    t = np.tanh(GELU_C * (z + GELU_A * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * z * z)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    return [(theta[w].reshape(shape), theta[b]) for w, shape, b in layer_slices()]


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def features(robot, q, qd, target):
    """x in R^21 from the state and the pose target (the force target and the
    wall are not inputs)."""
    qmax = np.array([L["q_max"] for L in robot["links"]], dtype=np.float64)
    qdmax = np.array([L["qd_max"] for L in robot["links"]], dtype=np.float64)
    quat = np.asarray(target["quat_des"], dtype=np.float64)
    quat = quat / np.linalg.norm(quat)
    if quat[0] < 0:
        quat = -quat
    return np.concatenate([np.asarray(q, float) / qmax, np.asarray(qd, float) / qdmax,
                           np.asarray(target["p_des"], float), quat])


def torque_scale(robot):
    return np.array([L["tau_max"] for L in robot["links"]], dtype=np.float64)


def normalised_targets(robot, U):
    """y* [126] from a torque sequence U [18][7]."""
    return (np.asarray(U, dtype=np.float64) / torque_scale(robot)).ravel()


def torques(robot, y):
    """U [18][7] from a network output y [126]."""
    return np.asarray(y, dtype=np.float64).reshape(T_STEPS, NJ) * torque_scale(robot)


def forward(theta, X, mirror=True):
    """y [B][126] and the cache (a_0..a_3, z_1..z_3) for a batch X [B][21]."""
    rnd = bf16 if mirror else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(theta)
    a = rnd(np.atleast_2d(np.asarray(X, dtype=np.float64)))
    acts, zs = [a], []
    for li, (W, b) in enumerate(layers):
        z = a @ rnd(W).T + b
        if li == 3:
            return z, (acts, zs)
        zs.append(z)
        a = rnd(gelu(z))
        acts.append(a)


def loss_and_grad(theta, X, Y, mirror=True):
    """L and dL/dtheta (flat) for a batch X [B][21], Y [B][126]."""
    rnd = bf16 if mirror else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(theta)
    y, (acts, zs) = forward(theta, X, mirror)
    Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
    B = y.shape[0]
    r = y - Y
    L = float(np.sum(r * r) / (B * DIMS[-1]))
    e = rnd(2.0 * r / (B * DIMS[-1]))
    grads = [None] * 4
    for li in range(3, -1, -1):
        W, _ = layers[li]
        grads[li] = (e.T @ acts[li], e.sum(axis=0))
        if li > 0:
            e = rnd((e @ rnd(W)) * gelu_prime(zs[li - 1]))
    return L, pack(grads)


def adam(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t = 1, 2, ...); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
