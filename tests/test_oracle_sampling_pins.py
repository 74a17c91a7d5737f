"""Pins of the oracle's sampling variants: temporally correlated (AR(1))
noise and several MPPI iterations per call."""
import numpy as np
import pytest


def test_rho_zero_is_the_iid_noise(ora, workloads):
    case = workloads["single_k256"][0]
    cost = dict(case["cost"], K=8)
    _, _, _, E = ora.update(case["robot"], cost, case["target"], case["q0"], case["qd0"], case["U_nom"], 5, 3)
    sig = np.asarray(cost["sigma"])
    for k in range(8):
        for t in range(cost["T"]):
            assert np.array_equal(E[k, t], sig * ora.normals(5, 3, k, t)[:7])


def test_ar1_noise_statistics(ora, workloads):
    """Stationary AR(1): variance sigma^2 at every step, lag-l correlation
    rho^l (estimates over 20,000 samples)."""
    case = workloads["single_k256"][1]
    rho = 0.8
    cost = dict(case["cost"], K=20000, T=6, noise_rho=rho)
    U = np.asarray(case["U_nom"])[:6]
    _, _, _, E = ora.update(case["robot"], cost, case["target"], case["q0"], case["qd0"], U, 9, 1)
    sig = np.asarray(cost["sigma"])
    x = E / sig                      # unit-variance process per joint
    for t in range(6):
        assert np.var(x[:, t, :]) == pytest.approx(1.0, abs=0.03)
    for lag in (1, 2, 3):
        c = np.mean([np.corrcoef(x[:, 2, j], x[:, 2 + lag, j])[0, 1] for j in range(7)])
        assert c == pytest.approx(rho ** lag, abs=0.02)
    # the recursion itself on one sample, from its normals
    k = 17
    z = np.array([ora.normals(9, 1, k, t)[:7] for t in range(6)])
    d = sig * z[0]
    assert np.allclose(E[k, 0], d, rtol=1e-15, atol=0)
    for t in range(1, 6):
        d = rho * d + np.sqrt(1 - rho * rho) * sig * z[t]
        assert np.allclose(E[k, t], d, rtol=1e-14, atol=1e-15)


def test_iterations_chain_updates(ora, workloads):
    """K = 1: each iteration adds its own sample exactly (Eq. 4b with one
    sample), iteration i drawing with Philox tick iterations * tick + i;
    one iteration is the plain update."""
    case = workloads["single_k256"][2]
    cost = dict(case["cost"], K=1, iterations=3)
    U0 = np.asarray(case["U_nom"])
    st, U, _, _ = ora.update(case["robot"], cost, case["target"], case["q0"], case["qd0"], U0, 4, 7)
    assert st == 0
    sig = np.asarray(cost["sigma"])
    add = sum(sig * np.array([ora.normals(4, 3 * 7 + i, 0, t)[:7] for t in range(cost["T"])]) for i in range(3))
    assert np.allclose(U, U0 + add, rtol=0, atol=1e-12)
    st1, U1, S1, _ = ora.update(case["robot"], dict(case["cost"], iterations=1), case["target"], case["q0"],
                                case["qd0"], U0, 4, 7)
    st0, U0b, S0, _ = ora.update(case["robot"], case["cost"], case["target"], case["q0"], case["qd0"], U0, 4, 7)
    assert np.array_equal(U1, U0b) and np.array_equal(S1, S0)


def test_iterations_are_chained_single_updates(ora, workloads):
    """n iterations at tick t are n single updates at the ticks n t + i, each
    from the previous U_new (structure of the chaining, K = 256)."""
    case = workloads["single_k256"][4]
    n, t = 3, 4
    st, U_n, S_n, E_n = ora.update(case["robot"], dict(case["cost"], iterations=n), case["target"], case["q0"],
                                   case["qd0"], case["U_nom"], 2, t)
    U = np.asarray(case["U_nom"])
    for i in range(n):
        st, U, S, E = ora.update(case["robot"], case["cost"], case["target"], case["q0"], case["qd0"], U, 2,
                                 n * t + i)
    assert np.array_equal(U, U_n) and np.array_equal(S, S_n) and np.array_equal(E, E_n)
