"""Pins for the oracle's Algorithm 1 (Sec. IV) and its derivative: brute force
on tiny tables, affine reproduction, continuity, finite differences, and the
partition of unity of the hat functions."""

import math

import numpy as np

import oracle as O


def brute_eval(X, v, x):
    """Algorithm 1 with a linear scan and Python floats, plus the clamping
    and end-point conventions of the oracle."""
    N = len(X) - 1
    if math.isnan(x):
        return float("nan"), -1
    x = min(max(x, X[0]), X[N])
    i = 0
    for k in range(1, N):
        if X[k] <= x:
            i = k
    d = (x - X[i]) / (X[i + 1] - X[i])
    return (1.0 - d) * v[i] + d * v[i + 1], i


def _tiny_tables():
    rng = np.random.default_rng(11)
    for N in (1, 2, 3, 5, 8):
        X = np.sort(rng.uniform(-3, 3, N + 1))
        X = O.fl32(X)
        if np.any(np.diff(X) <= 0):
            continue
        v = rng.standard_normal(N + 1)
        yield X, v


def test_eval_brute_force_on_tiny_tables():
    rng = np.random.default_rng(12)
    for X, v in _tiny_tables():
        pts = list(rng.uniform(X[0] - 1, X[-1] + 1, 200)) + list(X) + [X[0] - 5, X[-1] + 5, float("nan")]
        pts = list(O.fl32(np.array(pts)))
        y = O.evaluate(X, v, np.array(pts))
        idx = O.locate(X, np.array(pts))
        for p, yy, ii in zip(pts, y, idx):
            yb, ib = brute_eval(X, v, p)
            if math.isnan(p):
                assert math.isnan(yy)
                continue
            assert ii == ib
            assert abs(yy - yb) <= 1e-15 * max(1.0, np.abs(v).max())


def test_knot_points_go_right_and_ends_clamp():
    X = np.array([-1.0, 0.0, 0.5, 2.0])
    v = np.array([3.0, -1.0, 4.0, 1.0])
    assert list(O.locate(X, np.array([-1.0, 0.0, 0.5, 2.0, -7.0, 9.0]))) == [0, 1, 2, 2, 0, 2]
    y = O.evaluate(X, v, np.array([-1.0, 0.0, 0.5, 2.0, -7.0, 9.0]))
    assert list(y) == [3.0, -1.0, 4.0, 1.0, 3.0, 1.0]


def test_affine_table_is_exact():
    X, _, _ = O.optimal_knots(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 100)
    v = 2.5 - 0.75 * X
    x = np.linspace(-5.0, 5.0, 10001)
    assert np.max(np.abs(O.evaluate(X, v, x) - (2.5 - 0.75 * x))) <= 4e-15


def test_eval_is_continuous_at_knots():
    tb = O.build_table(O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 64, O.OPTIMAL, O.PROJ)
    X, v = tb["X"], tb["v"]
    left = O.evaluate(X, v, np.nextafter(X[1:-1], -np.inf))
    at = O.evaluate(X, v, X[1:-1])
    assert np.max(np.abs(left - at)) <= 1e-12
    assert np.array_equal(at, v[1:-1])


def test_backward_matches_finite_differences_in_x():
    tb = O.build_table(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 32, O.OPTIMAL, O.PROJ)
    X, v = tb["X"], tb["v"]
    rng = np.random.default_rng(4)
    x = rng.uniform(-5.5, 5.5, 500)
    g = rng.standard_normal(500)
    y, dx, dv = O.evaluate_backward(X, v, x, g)
    eps = 1e-7
    gap = np.min(np.abs(x[:, None] - X[None, :]), axis=1)
    ok = gap > 4 * eps
    fd = (O.evaluate(X, v, x + eps) - O.evaluate(X, v, x - eps)) / (2 * eps) * g
    assert np.max(np.abs(dx[ok] - fd[ok])) <= 1e-6 * np.max(np.abs(g))
    assert np.all(dx[(x < -5.0) | (x > 5.0)] == 0.0)


def test_backward_values_gradient_is_exact_by_linearity():
    # y is linear in v, so a finite difference in v_k is exact up to rounding.
    tb = O.build_table(O.BESSEL_J0, (1.0,), 0.0, 50.0, 20, O.OPTIMAL, O.INTERP)
    X, v = tb["X"], tb["v"]
    rng = np.random.default_rng(9)
    x = rng.uniform(-1.0, 51.0, 300)
    g = rng.standard_normal(300)
    _, _, dv = O.evaluate_backward(X, v, x, g)
    for k in range(len(v)):
        e = np.zeros_like(v)
        e[k] = 1.0
        fd = np.sum(g * (O.evaluate(X, v + e, x) - O.evaluate(X, v, x)))
        assert abs(dv[k] - fd) <= 1e-12 * np.sum(np.abs(g))


def test_backward_partition_of_unity_and_nan():
    X = O.fl32(np.array([0.0, 0.3, 1.1, 2.0]))
    v = np.array([1.0, 2.0, 0.0, -1.0])
    x = O.fl32(np.array([-1.0, 0.0, 0.3, 0.7, 2.0, 3.0, float("nan")]))
    g = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0])
    y, dx, dv = O.evaluate_backward(X, v, x, g)
    assert math.isclose(dv.sum(), g[:-1].sum(), rel_tol=1e-15)
    assert math.isnan(y[-1]) and math.isnan(dx[-1])
    assert dx[0] == 0.0 and dx[5] == 0.0
    assert dx[4] == 5.0 * (v[3] - v[2]) / (X[3] - X[2])   # left slope at b
    assert dv[0] == 1.0 + 2.0 and dv[3] >= 6.0


def test_backward_brute_force_scatter():
    rng = np.random.default_rng(21)
    for X, v in _tiny_tables():
        x = O.fl32(rng.uniform(X[0] - 0.5, X[-1] + 0.5, 64))
        g = rng.standard_normal(64)
        _, _, dv = O.evaluate_backward(X, v, x, g)
        ref = np.zeros(len(X))
        for p, gg in zip(x, g):
            _, i = brute_eval(X, v, p)
            pc = min(max(p, X[0]), X[-1])
            d = (pc - X[i]) / (X[i + 1] - X[i])
            ref[i] += (1 - d) * gg
            ref[i + 1] += d * gg
        assert np.max(np.abs(dv - ref)) <= 1e-13
