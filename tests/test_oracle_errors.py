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
