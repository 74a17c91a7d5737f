"""Pins of the oracle's warm start for solver periods that differ from the
horizon step (the mean of the piecewise-constant sequence over the shifted
step)."""
import numpy as np
import pytest


@pytest.fixture
def U():
    return np.random.default_rng(3).normal(size=(18, 7)) * 5


def test_one_step_is_the_usual_shift(ora, U):
    W = ora.warm_start(U, 1.0)
    assert np.array_equal(W[:-1], U[1:]) and np.array_equal(W[-1], U[-1])


@pytest.mark.parametrize("m", [0, 2, 5, 17, 18])
def test_integer_shifts(ora, U, m):
    W = ora.warm_start(U, float(m))
    idx = np.minimum(np.arange(18) + m, 17)
    assert np.array_equal(W, U[idx])


@pytest.mark.parametrize("s", [0.1, 0.6, 1.25, 3.999, 16.5])
def test_brute_force_mean_of_the_step_function(ora, U, s):
    """Midpoint-rule average of the held sequence over [t+s, t+s+1) on a
    fine grid (error below one grid cell times the largest jump)."""
    W = ora.warm_start(U, s)
    N = 20000
    x = (np.arange(N) + 0.5) / N
    for t in range(18):
        rows = np.minimum(np.floor(t + s + x).astype(int), 17)
        ref = U[rows].mean(axis=0)
        assert np.abs(W[t] - ref).max() <= 2.0 / N * np.abs(np.diff(U, axis=0)).max() + 1e-12


def test_ramp_and_constant(ora):
    """A ramp u_t = t (held) averages to t + s inside the horizon; a constant
    sequence stays constant."""
    R = np.tile(np.arange(18.0)[:, None], (1, 7))
    for s in (0.3, 0.75, 2.5):
        W = ora.warm_start(R, s)
        inside = np.arange(18) + s + 1 <= 17
        assert np.allclose(W[inside], (np.arange(18) + s)[inside][:, None], rtol=0, atol=1e-13)
        assert np.allclose(W[-1], R[-1], rtol=0, atol=1e-13)
    Cst = np.full((18, 7), 2.5)
    assert np.allclose(ora.warm_start(Cst, 0.37), Cst, rtol=0, atol=1e-14)


def test_linear_in_the_sequence(ora, U):
    V = np.random.default_rng(4).normal(size=U.shape)
    s = 0.42
    assert np.allclose(ora.warm_start(2 * U - 3 * V, s), 2 * ora.warm_start(U, s) - 3 * ora.warm_start(V, s),
                       rtol=0, atol=1e-12)
