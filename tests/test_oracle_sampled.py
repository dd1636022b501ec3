"""Pins of the oracle's sampled functions (the cubic spline with given values
and second derivatives) against closed forms: exact reproduction of a cubic
(inside and outside the sampled interval), the h^4 error of a smooth
function, exactness at the samples, and a table built from samples of the
Gaussian against the one built from the Gaussian itself."""

import numpy as np

import oracle as O


def _samples(f, f2, a, b, S):
    t = a + (b - a) * np.arange(S + 1) / S
    return O.Samples(f(t), f2(t), a, b)


def test_cubic_is_reproduced_exactly():
    c = np.array([1.0, 2.0, -0.5, 0.25])
    P = np.polynomial.polynomial
    for S in (1, 2, 7, 64):
        smp = _samples(lambda t: P.polyval(t, c), lambda t: P.polyval(t, P.polyder(c, 2)), -2.0, 3.0, S)
        x = np.linspace(-2.5, 3.5, 2001)
        assert np.max(np.abs(O.f_value(O.SAMPLED, smp, x) - P.polyval(x, c))) <= 1e-12
        assert np.max(np.abs(O.f_second(O.SAMPLED, smp, x) - P.polyval(x, P.polyder(c, 2)))) <= 1e-12


def test_smooth_function_error_is_fourth_order():
    g = lambda t: np.exp(-t * t / 2.0)
    g2 = lambda t: (t * t - 1.0) * np.exp(-t * t / 2.0)
    x = np.linspace(-5.0, 5.0, 100001)
    errs = []
    for S in (256, 512, 1024, 2048):
        h = 10.0 / S
        e = np.max(np.abs(O.f_value(O.SAMPLED, _samples(g, g2, -5.0, 5.0, S), x) - g(x)))
        assert e <= h ** 4 * 3.0 / 24.0          # max |g''''| = 3
        errs.append(e)
    slopes = np.diff(np.log(errs)) / np.diff(np.log([256, 512, 1024, 2048]))
    assert np.all(np.abs(slopes + 4.0) <= 0.3), slopes


def test_exact_at_the_samples():
    g = lambda t: np.sin(3 * t) * np.exp(-t * t / 4)
    g2 = lambda t: np.exp(-t * t / 4) * (-9 * np.sin(3 * t) - 3 * t * np.cos(3 * t) + (t * t / 4 - 0.5) * np.sin(3 * t))
    smp = _samples(g, g2, -6.0, 6.0, 300)
    t = -6.0 + 12.0 * np.arange(301) / 300
    # t_i recomputed from (t - a) / h lands within rounding of u = 0
    assert np.max(np.abs(O.f_value(O.SAMPLED, smp, t) - smp.f)) <= 1e-14
    assert np.max(np.abs(O.f_second(O.SAMPLED, smp, t) - smp.f2)) <= 1e-13


def test_table_from_samples_matches_table_from_function():
    g = lambda t: np.exp(-t * t / 2.0)
    g2 = lambda t: (t * t - 1.0) * np.exp(-t * t / 2.0)
    smp = _samples(g, g2, -5.0, 5.0, 1 << 14)
    for part in (O.UNIFORM, O.OPTIMAL):
        ts = O.build_table(O.SAMPLED, smp, -5.0, 5.0, 256, part, O.PROJ)
        tf = O.build_table(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 256, part, O.PROJ)
        x = np.linspace(-5.0, 5.0, 20001)
        d = np.max(np.abs(O.evaluate(ts["X"], ts["v"], x) - O.evaluate(tf["X"], tf["v"], x)))
        assert d <= 1e-7, (part, d)
