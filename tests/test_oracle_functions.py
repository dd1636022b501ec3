"""Pins for the oracle's function library: values and second derivatives are
checked against closed-form special values and against mpmath (30 digits),
which shares nothing with the oracle's formulas."""

import math

import mpmath
import numpy as np
import pytest

import oracle as O

mpmath.mp.dps = 30


def _mp_f(func, params):
    if func == O.GAUSSIAN:
        s, amp = params
        return lambda x: amp * mpmath.exp(-x * x / (2 * s * s))
    if func == O.LORENTZIAN:
        g, amp = params
        return lambda x: amp / (1 + (x / g) ** 2)
    if func == O.BESSEL_J0:
        (amp,) = params
        return lambda x: amp * mpmath.besselj(0, x)
    if func == O.POLY:
        return lambda x: sum(c * x ** k for k, c in enumerate(params))
    if func == O.EXP:
        al, amp = params
        return lambda x: amp * mpmath.exp(al * x)
    raise AssertionError


CASES = [
    (O.GAUSSIAN, (1.0, 1.0), [-4.9, -1.0, -0.3, 0.0, 0.7, 2.2, 4.0]),
    (O.GAUSSIAN, (0.37, 2.5), [-1.5, -0.2, 0.0, 0.37, 1.1]),
    (O.LORENTZIAN, (1.0, 1.0), [-19.0, -3.0, -0.5773, 0.0, 0.9, 7.5, 20.0]),
    (O.LORENTZIAN, (4.2, 0.5), [-60.0, -4.2, 0.0, 2.0, 33.0]),
    (O.BESSEL_J0, (1.0,), [0.0, 0.3, 2.404825557695773, 5.0, 13.7, 31.0, 49.9]),
    (O.POLY, (24.0, -20.0, -15.0, 5.0, 5.0, 1.0), [-4.0, -2.5, 0.0, 1.3, 3.0]),
    (O.EXP, (1.7, 0.4), [-2.0, 0.0, 1.0, 3.5]),
]


@pytest.mark.parametrize("func,params,xs", CASES)
def test_value_matches_mpmath(func, params, xs):
    ref = _mp_f(func, params)
    got = O.f_value(func, params, np.array(xs))
    for x, y in zip(xs, got):
        r = float(ref(mpmath.mpf(x)))
        # Polynomials cancel: scale the tolerance by the sum of |terms|.
        scale = sum(abs(c * x ** k) for k, c in enumerate(params)) if func == O.POLY else abs(r)
        assert abs(y - r) <= 4e-16 * max(1.0, scale), (x, y, r)


@pytest.mark.parametrize("func,params,xs", CASES)
def test_second_derivative_matches_mpmath(func, params, xs):
    ref = _mp_f(func, params)
    got = O.f_second(func, params, np.array(xs))
    for x, y in zip(xs, got):
        r = float(mpmath.diff(ref, mpmath.mpf(x), 2))
        assert abs(y - r) <= 1e-13 * max(1.0, abs(r)), (x, y, r)


def test_special_values():
    # Gaussian: f(0) = amp, f(s) = amp e^{-1/2}; f''(+-s) = 0.
    assert O.f_value(O.GAUSSIAN, (2.0, 3.0), 0.0) == 3.0
    assert math.isclose(O.f_value(O.GAUSSIAN, (2.0, 3.0), 2.0), 3.0 * math.exp(-0.5), rel_tol=1e-15)
    assert abs(O.f_second(O.GAUSSIAN, (2.0, 3.0), 2.0)) < 1e-16
    # Lorentzian: f(g) = amp/2, f''(0) = -2 amp / g^2, f'' = 0 at g/sqrt(3).
    assert O.f_value(O.LORENTZIAN, (2.0, 3.0), 2.0) == 1.5
    assert math.isclose(O.f_second(O.LORENTZIAN, (2.0, 3.0), 0.0), -1.5, rel_tol=1e-15)
    assert abs(O.f_second(O.LORENTZIAN, (1.0, 1.0), 1.0 / math.sqrt(3.0))) < 1e-15
    # J0: J0(0) = 1, J0''(0) = -1/2, first zero j_{0,1}.
    assert O.f_value(O.BESSEL_J0, (1.0,), 0.0) == 1.0
    assert math.isclose(O.f_second(O.BESSEL_J0, (1.0,), 0.0), -0.5, rel_tol=1e-15)
    assert abs(O.f_value(O.BESSEL_J0, (1.0,), 2.404825557695773)) < 1e-15
    # Affine functions have f'' == 0.
    assert np.all(O.f_second(O.POLY, (1.0, 2.0), np.linspace(-3, 3, 11)) == 0.0)


def test_density_is_two_fifths_power(golden_dir):
    from tests.golden_util import paper_constants
    e = paper_constants(golden_dir)["density_exponent"]
    x = np.array([-3.0, -0.4, 0.25, 2.0])
    d = O.density(O.GAUSSIAN, (1.0, 1.0), x)
    assert np.allclose(d, np.abs(O.f_second(O.GAUSSIAN, (1.0, 1.0), x)) ** e, rtol=1e-15)
