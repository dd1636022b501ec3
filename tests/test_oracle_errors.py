"""Pins for the oracle's error measures against the paper's error analysis:
exact closed forms for quadratics (Appendix A and B), the rigorous Result 1
bound, and the asymptotic Results 4-6 with a tolerance schedule in N."""

import math

import numpy as np
import pytest

import oracle as O


@pytest.fixture(scope="module")
def const(golden_dir):
    from tests.golden_util import paper_constants
    return paper_constants(golden_dir)


@pytest.mark.parametrize("partition", [O.UNIFORM, O.OPTIMAL])
def test_quadratic_interpolant_error_is_exact(const, partition):
    # eq. (SquaredErrorLinInterp) with f'' constant: the squared L2 error is
    # exactly sum_i h_i^5 f''^2 / 120 on any partition.
    p = (1.0, 0.5, -0.9)   # f'' = -1.8
    if partition == O.UNIFORM:
        X, _ = O.uniform_knots(-3.0, 2.0, 37)
    else:
        X, _, _ = O.optimal_knots(O.GAUSSIAN, (1.0, 1.0), -3.0, 2.0, 37)   # any non-uniform knots
    v = O.interp_values(O.POLY, p, X)
    h = np.diff(X)
    exact = np.sum(h ** 5) * 1.8 ** 2 / const["interp_sq_err_denominator"]
    assert math.isclose(O.l2_error(O.POLY, p, X, v) ** 2, exact, rel_tol=1e-12)


def test_quadratic_uniform_projection_error_is_exact(const):
    # Corollary of Result 2 with f'' constant, and P_T f equal to the union of
    # best segments on a uniform partition: ||f - P f||^2 = N h^5 f''^2 / 720.
    p = (0.2, 0.0, 2.0)    # f'' = 4
    N = 25
    X, _ = O.uniform_knots(-1.0, 4.0, N)
    h = 5.0 / N
    c = O.proj_values(O.POLY, p, X)
    exact = N * h ** 5 * 16.0 / const["best_segment_sq_err_denominator"]
    assert math.isclose(O.l2_error(O.POLY, p, X, c) ** 2, exact, rel_tol=1e-11)


def test_quadratic_projection_error_bracket_nonuniform(const):
    # For f'' constant on any partition, the best single segments give the
    # lower bound sum h^5 f''^2 / 720 and the interpolant the upper bound
    # sum h^5 f''^2 / 120.
    p = (0.0, 1.0, 1.5)
    X, _, _ = O.optimal_knots(O.LORENTZIAN, (1.0, 1.0), -4.0, 4.0, 31)
    h = np.diff(X)
    e2 = O.l2_error(O.POLY, p, X, O.proj_values(O.POLY, p, X)) ** 2
    s = np.sum(h ** 5) * 9.0
    assert s / const["best_segment_sq_err_denominator"] * (1 - 1e-12) <= e2
    assert e2 <= s / const["interp_sq_err_denominator"]


def test_best_single_segment_matches_result2_for_quadratic(const):
    # Result 2 with f'' = k constant: min error^2 = h^5 k^2 (1/120 - 1/144),
    # which is h^5 k^2 / 720 (the Corollary).
    k, h = 3.0, 0.7
    exact = h ** 5 * k * k * (1.0 / const["interp_sq_err_denominator"]
                              - 1.0 / const["best_segment_correction_denominator"])
    assert math.isclose(exact, h ** 5 * k * k / const["best_segment_sq_err_denominator"], rel_tol=1e-14)
    X = np.array([0.0, h])
    p = (0.0, 0.0, k / 2.0)
    c = O.proj_values(O.POLY, p, X)
    assert math.isclose(O.l2_error(O.POLY, p, X, c) ** 2, exact, rel_tol=1e-11)


@pytest.mark.parametrize("func,p,a,b", [
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0),
])
@pytest.mark.parametrize("N", [16, 64, 256])
def test_result1_rigorous_bound(func, p, a, b, N):
    for part in (O.UNIFORM, O.OPTIMAL):
        tb = O.build_table(func, p, a, b, N, part, O.INTERP)
        err = O.l2_error(func, p, tb["X"], tb["v"])
        assert err <= O.result1_bound(func, p, tb["X"]) * (1 + 1e-3)
        # the projection can only be closer (eq. phf-is-the-best)
        tp = O.build_table(func, p, a, b, N, part, O.PROJ)
        assert O.l2_error(func, p, tp["X"], tp["v"]) <= err


FUNCS = [
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0),
]


@pytest.mark.parametrize("func,p,a,b", FUNCS)
def test_asymptotic_results_4_5_6(func, p, a, b):
    # Results 4-6 are asymptotic.  Schedule: |measured/predicted - 1| <= 5% at
    # N = 256 and <= 1% at N >= 1024; the projection/interpolant ratio is
    # 1/sqrt(6) within 2% at N >= 1024 (Result 5).
    for N, tol in ((256, 0.05), (1024, 0.01), (4096, 0.01)):
        pe = O.predicted_errors(func, p, a, b, N)
        errs = {}
        for part in (O.UNIFORM, O.OPTIMAL):
            for val in (O.INTERP, O.PROJ):
                tb = O.build_table(func, p, a, b, N, part, val)
                errs[(part, val)] = O.l2_error(func, p, tb["X"], tb["v"])
                ratio = errs[(part, val)] / pe["l2"][(part, val)]
                assert abs(ratio - 1.0) <= tol, (N, part, val, ratio)
        if N >= 1024:
            for part in (O.UNIFORM, O.OPTIMAL):
                r = math.sqrt(6.0) * errs[(part, O.PROJ)] / errs[(part, O.INTERP)]
                assert abs(r - 1.0) <= 0.02, (N, part, r)
        # the optimised partition never loses to the uniform one here
        assert errs[(O.OPTIMAL, O.INTERP)] <= errs[(O.UNIFORM, O.INTERP)]


@pytest.mark.parametrize("func,p,a,b", FUNCS)
def test_linf_predictions(func, p, a, b):
    N = 1024
    pe = O.predicted_errors(func, p, a, b, N)
    for part in (O.UNIFORM, O.OPTIMAL):
        for val in (O.INTERP, O.PROJ):
            tb = O.build_table(func, p, a, b, N, part, val)
            r = O.linf_error(func, p, tb["X"], tb["v"]) / pe["linf"][(part, val)]
            assert abs(r - 1.0) <= 0.05, (part, val, r)


@pytest.mark.parametrize("func,p,a,b", FUNCS)
def test_convergence_order_two(func, p, a, b, const):
    order = const["convergence_order"]
    Ns = [256, 512, 1024, 2048]
    for part in (O.UNIFORM, O.OPTIMAL):
        for val in (O.INTERP, O.PROJ):
            e = [O.l2_error(func, p, *(lambda t: (t["X"], t["v"]))(O.build_table(func, p, a, b, N, part, val)))
                 for N in Ns]
            slopes = np.diff(np.log(e)) / np.diff(np.log(Ns))
            assert np.all(np.abs(slopes + order) <= 0.05), (part, val, slopes)


# ---------------------------------------------------------------------------
# Exact pins of linf_error and result1_bound (closed forms for polynomials).
# ---------------------------------------------------------------------------

def _random_partition(a, b, N, seed):
    rng = np.random.default_rng(seed)
    inner = np.sort(rng.uniform(a, b, N - 1))
    return np.concatenate([[a], inner, [b]])


def test_linf_interpolant_of_quadratic_is_max_h2_over_8():
    # f = c x^2 / 2 has f'' = c; on [x_i, x_{i+1}] the interpolation error is
    # (c/2)(x - x_i)(x_{i+1} - x), largest at the midpoint: c h_i^2 / 8
    # (the interpolation remainder, Appendix A).
    c = 2.6
    X = _random_partition(-3.0, 5.0, 23, 11)
    p = (0.4, -1.1, c / 2.0)
    v = O.interp_values(O.POLY, p, X)
    exact = c * np.max(np.diff(X)) ** 2 / 8.0
    assert math.isclose(O.linf_error(O.POLY, p, X, v), exact, rel_tol=1e-12)


def test_linf_uniform_projection_of_quadratic_is_h2_over_12():
    # On a uniform partition the projection of c x^2/2 is the interpolant
    # lowered by c h^2 / 12 on every segment (the per-segment minimiser of
    # Appendix B, continuous because every h is equal): the error is c h^2/12
    # at the knots and -c h^2/24 at the midpoints, so the maximum is c h^2/12.
    # N = 32 on [-2, 6]: h = 1/4, so the FP32 knots are exactly uniform.
    c, N = 3.0, 32
    X, _ = O.uniform_knots(-2.0, 6.0, N)
    h = 8.0 / N
    assert np.all(np.diff(X) == h)
    p = (0.0, 0.7, c / 2.0)
    cv = O.proj_values(O.POLY, p, X)
    assert math.isclose(O.linf_error(O.POLY, p, X, cv), c * h * h / 12.0, rel_tol=1e-10)


def _cubic_interp_linf_exact(p, X):
    """max |f - pi f| for f = c0 + c1 x + c2 x^2 + c3 x^3, in closed form: on
    a segment, with u = x - x_i and h = x_{i+1} - x_i, the error is
    e(u) = u (u - h) (A + c3 u), A = c2 + c3 (2 x_i + x_{i+1}) (the second
    divided difference of a cubic); its extrema solve the quadratic e'(u) = 0."""
    c2, c3 = p[2], p[3]
    best = 0.0
    for x0, x1 in zip(X[:-1], X[1:]):
        h = x1 - x0
        A = c2 + c3 * (2.0 * x0 + x1)
        B = c3
        qa, qb, qc = 3.0 * B, 2.0 * (A - B * h), -A * h
        roots = [-qc / qb] if qa == 0.0 else []
        if qa != 0.0:
            disc = qb * qb - 4.0 * qa * qc
            if disc >= 0.0:
                r = math.sqrt(disc)
                roots = [(-qb - r) / (2.0 * qa), (-qb + r) / (2.0 * qa)]
        for u in roots:
            if 0.0 <= u <= h:
                best = max(best, abs(u * (u - h) * (A + B * u)))
    return best


def test_linf_interpolant_of_cubic_between_samples():
    # The maximum of a cubic's interpolation error does not sit on the 33
    # sample points of a segment, so this pins the golden-section refinement
    # as well as the sampling.
    p = (0.3, -0.2, 0.45, -0.37)
    X = _random_partition(-2.5, 3.0, 17, 5)
    v = O.interp_values(O.POLY, p, X)
    exact = _cubic_interp_linf_exact(p, X)
    got = O.linf_error(O.POLY, p, X, v)
    assert math.isclose(got, exact, rel_tol=1e-10)
    # the samples alone fall measurably short of it
    s = np.linspace(0.0, 1.0, 33)
    h = np.diff(X)
    xs = X[:-1, None] + h[:, None] * s[None, :]
    line = v[:-1, None] * (1.0 - s[None, :]) + v[1:, None] * s[None, :]
    sampled = float(np.max(np.abs(O.f_value(O.POLY, p, xs) - line)))
    assert sampled < exact * (1.0 - 1e-6)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_result1_bound_equals_error_for_quadratics(seed):
    # Result 1 (Sec. III-A) is an equality when f'' is constant: the bound
    # sqrt(sum_i max|f''|^2 h_i^5 / 120) is then the interpolant's L2 error.
    rng = np.random.default_rng(seed)
    p = tuple(rng.uniform(-2.0, 2.0, 3))
    X = _random_partition(-1.0, 4.0, 29, 20 + seed)
    err = O.l2_error(O.POLY, p, X, O.interp_values(O.POLY, p, X))
    assert math.isclose(O.result1_bound(O.POLY, p, X), err, rel_tol=1e-12)


def test_result1_bound_and_l2_error_of_cubic_in_closed_form():
    # For a cubic, f'' is linear, so its maximum on a segment is at an end:
    # the bound is sqrt(sum_i max(|f''(x_i)|, |f''(x_{i+1})|)^2 h_i^5 / 120).
    # The squared L2 error is the exact integral of the polynomial e(u)^2.
    p = (0.1, 0.5, -0.8, 0.6)
    X = _random_partition(-2.0, 2.0, 13, 9)
    f2 = lambda x: 2.0 * p[2] + 6.0 * p[3] * x
    h = np.diff(X)
    m = np.maximum(np.abs(f2(X[:-1])), np.abs(f2(X[1:])))
    assert math.isclose(O.result1_bound(O.POLY, p, X), math.sqrt(float(np.sum(m * m * h ** 5 / 120.0))),
                        rel_tol=1e-12)
    from numpy.polynomial import polynomial as Pn
    total = 0.0
    for x0, x1 in zip(X[:-1], X[1:]):
        hh = x1 - x0
        A = p[2] + p[3] * (2.0 * x0 + x1)
        e = Pn.polymul(Pn.polymul([0.0, 1.0], [-hh, 1.0]), [A, p[3]])   # u (u - h) (A + c3 u)
        sq = Pn.polyint(Pn.polymul(e, e))
        total += Pn.polyval(hh, sq) - Pn.polyval(0.0, sq)
    v = O.interp_values(O.POLY, p, X)
    assert math.isclose(O.l2_error(O.POLY, p, X, v) ** 2, total, rel_tol=1e-11)
