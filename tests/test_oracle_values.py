"""Pins for the oracle's vertex values: the interpolant (Sec. II-B1) and the
L2 projection (Sec. II-B2).  The projection is checked against independent
routes: adaptive quadrature for the Gram matrix and b with a dense solve, the
orthogonality condition, closed forms for b, the uniform-quadratic closed form
that follows from the minimisers of Appendix B, the N = 1 Legendre line, and
the best-approximation property."""

import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import erf

import oracle as O


def hat(X, k, x):
    """phi_k(x) written directly from its definition in Sec. II-B."""
    N = len(X) - 1
    if k > 0 and X[k - 1] <= x <= X[k]:
        return (x - X[k - 1]) / (X[k] - X[k - 1])
    if k < N and X[k] <= x <= X[k + 1]:
        return (x - X[k + 1]) / (X[k] - X[k + 1])
    return 0.0


def test_interp_values_are_f_at_fp32_knots():
    tb = O.build_table(O.BESSEL_J0, (1.0,), 0.0, 50.0, 256, O.OPTIMAL, O.INTERP)
    X = tb["X"]
    assert np.all(X == X.astype(np.float32))
    assert np.array_equal(tb["v"], O.f_value(O.BESSEL_J0, (1.0,), X))


@pytest.mark.parametrize("partition", [O.UNIFORM, O.OPTIMAL])
@pytest.mark.parametrize("values", [O.INTERP, O.PROJ])
def test_affine_function_is_reproduced(partition, values):
    # An affine f lies in V_T, so pi_T f = P_T f = f (Sec. II-B).
    p = (0.75, -1.25)
    tb = O.build_table(O.POLY, p, -3.0, 5.0, 33, partition, values)
    assert np.max(np.abs(tb["v"] - O.f_value(O.POLY, p, tb["X"]))) <= 1e-13


@pytest.mark.parametrize("N", [1, 2, 8, 16, 64])   # FP32-exact uniform knots
def test_uniform_quadratic_projection_closed_form(N, golden_dir):
    # Appendix B: with f'' constant, the best segment moves both ends by
    # (f'' - 2 f'') h^2 / 12 = -f'' h^2 / 12.  On a uniform partition these
    # shifts agree at every knot, so the best segments join continuously and
    # their union is P_T f: c_i = f(x_i) - f'' h^2 / 12 at every node.
    from tests.golden_util import paper_constants
    den = paper_constants(golden_dir)["minimiser_denominator"]
    p = (0.3, -0.7, 1.9)   # f'' = 3.8
    X, _ = O.uniform_knots(-2.0, 2.0, N)
    h = 4.0 / N
    c = O.proj_values(O.POLY, p, X)
    exact = O.f_value(O.POLY, p, X) - 3.8 * h * h / den
    assert np.max(np.abs(c - exact)) <= 1e-13


def test_single_segment_projection_is_legendre_line():
    # N = 1: V_T is the space of lines, so P_T f is the L2-best line, which is
    # the Legendre expansion truncated after degree one.
    for func, p, a, b in [(O.GAUSSIAN, (1.0, 1.0), -1.0, 2.0), (O.BESSEL_J0, (1.0,), 0.0, 6.0)]:
        X, _ = O.uniform_knots(a, b, 1)
        c = O.proj_values(func, p, X)
        mid, half = (a + b) / 2.0, (b - a) / 2.0
        m0 = quad(lambda x: float(O.f_value(func, p, x)), a, b, epsabs=0, epsrel=1e-13)[0] / (b - a)
        m1 = 3.0 * quad(lambda x: float(O.f_value(func, p, x)) * (x - mid) / half, a, b,
                        epsabs=0, epsrel=1e-13)[0] / (b - a)
        assert abs(c[0] - (m0 - m1)) <= 1e-12 and abs(c[1] - (m0 + m1)) <= 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 5, 8])
def test_projection_matches_dense_gram_solve(N):
    # The Gram matrix and b by adaptive quadrature of the hat functions as
    # defined in Sec. II-B, then a dense LU solve.
    func, p = O.GAUSSIAN, (0.8, 1.3)
    X, _, _ = O.optimal_knots(func, p, -2.5, 3.0, N)
    G = np.zeros((N + 1, N + 1))
    rhs = np.zeros(N + 1)
    for i in range(N + 1):
        lo, hi = X[max(i - 1, 0)], X[min(i + 1, N)]
        rhs[i] = quad(lambda x: float(O.f_value(func, p, x)) * hat(X, i, x), lo, hi,
                      points=[X[i]], epsabs=0, epsrel=1e-13)[0]
        for j in range(max(i - 1, 0), min(i + 1, N) + 1):
            G[i, j] = quad(lambda x: hat(X, i, x) * hat(X, j, x), lo, hi, points=[X[i]],
                           epsabs=0, epsrel=1e-13)[0]
    c_dense = np.linalg.solve(G, rhs)
    c = O.proj_values(func, p, X)
    # The oracle integrates b with 16-point Gauss-Legendre per segment; on the
    # single 5.5-wide segment of N = 1 that rule is only good to about 1e-11.
    assert np.max(np.abs(c - c_dense)) <= (5e-11 if N == 1 else 1e-12)


@pytest.mark.parametrize("func,p,a,b,N", [
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 16),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 16),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 24),
])
def test_projection_residual_is_orthogonal_to_every_hat(func, p, a, b, N):
    # eq. (phf): <f - P_T f, v> = 0 for all v in V_T; check it for each hat
    # with adaptive quadrature and the oracle's own evaluator for P_T f.
    tb = O.build_table(func, p, a, b, N, O.OPTIMAL, O.PROJ)
    X, v = tb["X"], tb["v"]
    scale = max(abs(float(O.f_value(func, p, 0.5 * (a + b)))), 1.0) * (b - a) / N
    for k in range(N + 1):
        lo, hi = X[max(k - 1, 0)], X[min(k + 1, N)]
        r = quad(lambda x: (float(O.f_value(func, p, x)) - float(O.evaluate(X, v, x))) * hat(X, k, x),
                 lo, hi, points=[X[k]], epsabs=1e-16, epsrel=1e-12, limit=200)[0]
        assert abs(r) <= 1e-11 * scale, (k, r)


def test_gaussian_hat_products_closed_form():
    # Integral of e^{-x^2/2} (x - c) dx = -e^{-x^2/2} - c sqrt(pi/2) erf(x/sqrt 2)
    # gives <f, phi_k> exactly for the unit Gaussian.
    X, _, _ = O.optimal_knots(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 40)
    N = len(X) - 1

    def prim(x, c):
        return -math.exp(-x * x / 2.0) - c * math.sqrt(math.pi / 2.0) * erf(x / math.sqrt(2.0))
    ref = np.zeros(N + 1)
    for k in range(N):
        x0, x1 = X[k], X[k + 1]
        h = x1 - x0
        # phi_k = (x1 - x)/h and phi_{k+1} = (x - x0)/h on [x0, x1]
        ref[k] += -(prim(x1, x1) - prim(x0, x1)) / h
        ref[k + 1] += (prim(x1, x0) - prim(x0, x0)) / h
    b = O.hat_inner_products(O.GAUSSIAN, (1.0, 1.0), X)
    assert np.max(np.abs(b - ref)) <= 2e-14


def test_lorentzian_hat_products_closed_form():
    # Integral of (x - c)/(1 + x^2) dx = ln(1 + x^2)/2 - c atan(x).
    X, _, _ = O.optimal_knots(O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 40)
    N = len(X) - 1

    def prim(x, c):
        return 0.5 * math.log1p(x * x) - c * math.atan(x)
    ref = np.zeros(N + 1)
    for k in range(N):
        x0, x1 = X[k], X[k + 1]
        h = x1 - x0
        ref[k] += -(prim(x1, x1) - prim(x0, x1)) / h
        ref[k + 1] += (prim(x1, x0) - prim(x0, x0)) / h
    b = O.hat_inner_products(O.LORENTZIAN, (1.0, 1.0), X)
    assert np.max(np.abs(b - ref)) <= 1e-12


def test_projection_is_best_approximation():
    # eq. (phf-is-the-best): any other w in V_T is farther from f.
    func, p = O.BESSEL_J0, (1.0,)
    tb = O.build_table(func, p, 0.0, 50.0, 48, O.OPTIMAL, O.PROJ)
    ti = O.build_table(func, p, 0.0, 50.0, 48, O.OPTIMAL, O.INTERP)
    X, c = tb["X"], tb["v"]
    e0 = O.l2_error(func, p, X, c)
    assert e0 < O.l2_error(func, p, ti["X"], ti["v"])
    rng = np.random.default_rng(5)
    for k in [0, 1, 17, 47, 48]:
        for eps in (1e-3, -1e-3, 1e-5):
            w = c.copy()
            w[k] += eps
            assert O.l2_error(func, p, X, w) > e0
    for _ in range(5):
        w = c + 1e-4 * rng.standard_normal(len(c))
        assert O.l2_error(func, p, X, w) > e0


def test_interpolant_lies_above_convex_stretches():
    # Sec. II-B1: pi_T f >= f wherever f is convex (Gaussian: |x| > 1).
    tb = O.build_table(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 64, O.OPTIMAL, O.INTERP)
    X, v = tb["X"], tb["v"]
    for k in range(64):
        if X[k] >= 1.0 or X[k + 1] <= -1.0:
            xs = np.linspace(X[k], X[k + 1], 41)
            assert np.all(O.evaluate(X, v, xs) - O.f_value(O.GAUSSIAN, (1.0, 1.0), xs) >= -1e-15)


def test_thomas_matches_dense_solve_on_random_dominant_systems():
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 10, 257):
        lo = rng.uniform(-1, 1, max(n - 1, 0))
        up = rng.uniform(-1, 1, max(n - 1, 0))
        di = np.abs(np.concatenate([[0.0], lo])) + np.abs(np.concatenate([up, [0.0]])) + rng.uniform(0.5, 2.0, n)
        A = np.diag(di) + np.diag(lo, -1) + np.diag(up, 1)
        r = rng.standard_normal(n)
        assert np.allclose(O.thomas(lo, di, up, r), np.linalg.solve(A, r), rtol=0, atol=1e-12)


def test_mass_matrix_matches_quadrature_of_hats():
    X = np.array([-1.0, -0.25, 0.5, 0.625, 2.0])
    lo, di, up = O.mass_matrix(X)
    N = 4
    for i in range(N + 1):
        a, b = X[max(i - 1, 0)], X[min(i + 1, N)]
        m = quad(lambda x: hat(X, i, x) ** 2, a, b, points=[X[i]], epsabs=0, epsrel=1e-13)[0]
        assert abs(di[i] - m) <= 1e-14
        if i < N:
            m = quad(lambda x: hat(X, i, x) * hat(X, i + 1, x), X[i], X[i + 1], epsabs=0, epsrel=1e-13)[0]
            assert abs(up[i] - m) <= 1e-14 and abs(lo[i] - m) <= 1e-14
