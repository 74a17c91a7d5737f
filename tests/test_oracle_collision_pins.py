"""Pins of the oracle's collision term (Eqs. 14-15): the segment distance
against an independent bounded minimiser and closed forms, the link
segments against forward kinematics, and the indicator count."""
import numpy as np
import pytest
from scipy.optimize import minimize


def brute_distance(a0, a1, b0, b1):
    """Bounded quasi-Newton minimisation of |a(s) - b(t)| over the unit
    square from a grid of starts (independent of the oracle's enumeration)."""
    a0, a1, b0, b1 = map(np.asarray, (a0, a1, b0, b1))
    f = lambda x: np.sum((a0 + x[0] * (a1 - a0) - b0 - x[1] * (b1 - b0)) ** 2)
    best = np.inf
    for s in (0.0, 0.5, 1.0):
        for t in (0.0, 0.5, 1.0):
            r = minimize(f, [s, t], bounds=[(0, 1), (0, 1)], method="L-BFGS-B", options={"ftol": 1e-15, "gtol": 1e-12})
            best = min(best, r.fun)
    return np.sqrt(best)


def test_segment_distance_matches_bounded_minimiser(ora):
    rng = np.random.default_rng(0)
    for _ in range(300):
        a0, a1, b0, b1 = rng.normal(size=(4, 3))
        assert ora.segment_distance(a0, a1, b0, b1) == pytest.approx(brute_distance(a0, a1, b0, b1), abs=1e-6)


def test_segment_distance_closed_forms(ora):
    # crossing segments
    assert ora.segment_distance([-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0]) == pytest.approx(0.0, abs=1e-15)
    # skew, closest points interior: |(b0 - a0) . (da x db)| / |da x db|
    a0, a1, b0, b1 = np.array([0., 0, 0]), np.array([2., 0, 0]), np.array([1., -1, 0.7]), np.array([1., 1, 0.7])
    n = np.cross(a1 - a0, b1 - b0)
    assert ora.segment_distance(a0, a1, b0, b1) == pytest.approx(abs((b0 - a0) @ n) / np.linalg.norm(n), rel=1e-14)
    # parallel, overlapping: the line distance; parallel, disjoint: end to end
    assert ora.segment_distance([0, 0, 0], [1, 0, 0], [0.5, 0.3, 0], [2, 0.3, 0]) == pytest.approx(0.3, rel=1e-14)
    assert ora.segment_distance([0, 0, 0], [1, 0, 0], [2, 0.3, 0], [3, 0.3, 0]) == pytest.approx(np.hypot(1, 0.3), rel=1e-14)
    # a zero-length segment is a point: point-to-segment distance
    assert ora.segment_distance([0.5, 2, 0], [0.5, 2, 0], [0, 0, 0], [1, 0, 0]) == pytest.approx(2.0, rel=1e-14)
    assert ora.segment_distance([3, 1, 0], [3, 1, 0], [0, 0, 0], [1, 0, 0]) == pytest.approx(np.hypot(2, 1), rel=1e-14)
    assert ora.segment_distance([1, 1, 1], [1, 1, 1], [1, 1, 1], [1, 1, 1]) == 0.0


def test_segment_distance_invariances(ora):
    rng = np.random.default_rng(1)
    from scipy.spatial.transform import Rotation
    for _ in range(50):
        a0, a1, b0, b1 = rng.normal(size=(4, 3))
        d = ora.segment_distance(a0, a1, b0, b1)
        assert ora.segment_distance(b0, b1, a0, a1) == pytest.approx(d, rel=1e-12, abs=1e-15)
        assert ora.segment_distance(a1, a0, b1, b0) == pytest.approx(d, rel=1e-12, abs=1e-15)
        R = Rotation.random(random_state=rng.integers(1 << 30)).as_matrix()
        x = rng.normal(size=3)
        assert ora.segment_distance(*(R @ p + x for p in (a0, a1, b0, b1))) == pytest.approx(d, rel=1e-10, abs=1e-12)


def test_link_segments_follow_forward_kinematics(ora, workloads):
    case = workloads["wall_k4096"][0]
    rb = case["robot"]
    q = np.asarray(case["q0"])
    seg = ora.link_segments(rb, q)
    _, p, pe, _ = ora.fk(rb, q)
    p = np.asarray(p).reshape(-1, 3)
    assert np.allclose(seg[:, :3], p, atol=0, rtol=0)
    assert np.allclose(seg[:-1, 3:], p[1:], atol=0, rtol=0)
    assert np.allclose(seg[-1, 3:], pe, atol=0, rtol=0)


def test_collision_indicator_counts_pairs_under_threshold(ora, workloads):
    case = workloads["wall_k4096"][0]
    rb = case["robot"]
    q = np.asarray(case["q0"])
    seg = ora.link_segments(rb, q)
    # an obstacle parallel to link 3 at 0.15 m, one at 0.5 m from every link
    a, b = seg[3, :3], seg[3, 3:]
    u = np.cross(b - a, [0.0, 0.0, 1.0])
    u /= np.linalg.norm(u)
    near = np.concatenate([a + 0.15 * u, b + 0.15 * u])
    cost = dict(case["cost"], w_collision=3e4, obstacles=[near.tolist()],
                pairs=[[3, 7], [3, 7], [0, 5]], d_th=[0.2, 0.1, 0.0])
    d = ora.segment_distance(seg[3, :3], seg[3, 3:], near[:3], near[3:])
    assert d <= 0.15 + 1e-12
    c, m = ora.collision_cost(rb, cost, q)
    d05 = ora.segment_distance(seg[0, :3], seg[0, 3:], seg[5, :3], seg[5, 3:])
    assert c == 3e4   # only the first pair is under its threshold
    assert m == pytest.approx(min(abs(d - 0.2), abs(d - 0.1), d05), rel=1e-12)
    total, parts = ora.running_cost(rb, cost, case["target"], q, case["qd0"], case["U_nom"][0])
    total0, parts0 = ora.running_cost(rb, dict(cost, pairs=[], d_th=[]), case["target"], q, case["qd0"],
                                      case["U_nom"][0])
    assert parts["collision"] == 3e4 and parts0["collision"] == 0.0
    assert total == pytest.approx(total0 + 3e4, rel=1e-15)
    # the rollout reports its closest approach to a threshold
    S, mr = ora.rollout_margin(rb, dict(cost, T=3), case["target"], q, case["qd0"], case["U_nom"][:3], 7, 0, 0)
    assert 0 <= mr <= m + 1e-9
