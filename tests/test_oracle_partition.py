"""Pins for the oracle's partitions (Sec. II-B uniform knots, Sec. III-B1
quasi-optimal knots): closed-form knot sets, symmetry, the exact-F cross-check
with adaptive quadrature plus root finding, and the degenerate cases."""

import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

import oracle as O


def ulp32(x):
    x = np.abs(np.asarray(x, dtype=np.float32))
    return (np.nextafter(x, np.float32(np.inf)) - x).astype(np.float64)


def test_uniform_knots_exact_eighths():
    X, X64 = O.uniform_knots(-4.0, 4.0, 64)
    assert np.array_equal(X, -4.0 + np.arange(65) / 8.0)
    assert X[0] == -4.0 and X[-1] == 4.0


def test_uniform_knots_are_rounded_equal_spacing():
    X, X64 = O.uniform_knots(-1.3, 2.9, 37)
    a, b = O.domain32(-1.3, 2.9)
    exact = a + (b - a) * np.arange(38) / 37.0
    assert np.all(np.abs(X - exact) <= 0.5 * ulp32(exact) + 1e-300)
    assert X[0] == a and X[-1] == b


@pytest.mark.parametrize("alpha,a,b,N", [(1.0, 0.0, 3.0, 64), (-2.5, -1.0, 2.0, 128), (0.7, -5.0, 5.0, 256)])
def test_optimal_knots_exponential_closed_form(alpha, a, b, N):
    # f = e^{alpha x}: |f''|^{2/5} = |alpha|^{4/5} e^{2 alpha x / 5}, so F is
    # explicit and x_i = a + 5/(2 alpha) ln(1 + (i/N)(e^{2 alpha (b-a)/5} - 1)).
    X, X64, flags = O.optimal_knots(O.EXP, (alpha, 1.0), a, b, N)
    assert flags == 0
    i = np.arange(N + 1)
    exact = a + 5.0 / (2.0 * alpha) * np.log1p((i / N) * math.expm1(2.0 * alpha * (b - a) / 5.0))
    assert np.max(np.abs(X64 - exact)) <= 1e-8 * (b - a)
    assert np.all(np.abs(X - exact) <= ulp32(exact) + 1e-8 * (b - a))


def test_optimal_knots_quartic_closed_form():
    # f = x^4/12 on [0, 1]: f'' = x^2, density x^(4/5), F(x) = x^(9/5),
    # x_i = (i/N)^(5/9).  The density has a cusp-free but non-smooth start at
    # 0 (x^0.8), so the trapezoid grid converges more slowly there.
    N = 50
    X, X64, flags = O.optimal_knots(O.POLY, (0, 0, 0, 0, 1.0 / 12.0), 0.0, 1.0, N)
    exact = (np.arange(N + 1) / N) ** (5.0 / 9.0)
    assert np.max(np.abs(X64 - exact)) <= 2e-6
    assert np.max(np.abs(X64 - exact)[5:]) <= 2e-8


def test_quadratic_gives_uniform_partition():
    # f'' constant => F linear => the quasi-optimal partition is uniform.
    X, X64, flags = O.optimal_knots(O.POLY, (0.5, -1.0, 3.0), -2.0, 7.0, 90)
    U, U64 = O.uniform_knots(-2.0, 7.0, 90)
    assert np.max(np.abs(X64 - U64)) <= 1e-12 * 9.0
    assert np.all(np.abs(X - U) <= ulp32(U))


@pytest.mark.parametrize("func,params,a,b,N", [
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 1024),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 256),
    (O.GAUSSIAN, (0.3, 2.0), -1.5, 1.5, 77),
])
def test_even_function_gives_symmetric_knots(func, params, a, b, N):
    X, X64, flags = O.optimal_knots(func, params, a, b, N)
    assert np.all(np.abs(X + X[::-1]) <= ulp32(X))
    if N % 2 == 0:
        assert X[N // 2] == 0.0


def _exact_F_knots(func, params, a, b, N, idx):
    zs = O.second_derivative_zeros(func, params, a, b)
    pts = [a] + zs + [b]

    def dens(z):
        return float(O.density(func, params, z))
    seg = [quad(dens, lo, hi, limit=400, epsabs=0, epsrel=1e-13)[0] for lo, hi in zip(pts[:-1], pts[1:])]
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    total = cum[-1]

    def F(x):
        k = int(np.searchsorted(pts, x, side="right") - 1)
        k = min(max(k, 0), len(seg) - 1)
        return cum[k] + quad(dens, pts[k], x, limit=400, epsabs=0, epsrel=1e-13)[0]
    out = []
    for i in idx:
        target = i * total / N
        out.append(brentq(lambda x: F(x) - target, a, b, xtol=1e-14, rtol=1e-15))
    return np.array(out)


@pytest.mark.parametrize("func,params,a,b,N", [
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 64),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 64),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 64),
])
def test_optimal_knots_match_exact_inverse_cdf(func, params, a, b, N):
    # Independent route to F^{-1}(i/N): adaptive quadrature of the density and
    # Brent root finding; the oracle's M = 256 N trapezoid grid must agree.
    # The density |f''|^(2/5) has |x - z|^(2/5) cusps at the zeros z of f'',
    # so the trapezoid grid converges like dt^(7/5) there: at M = 256 N the
    # knots sit within a few 1e-6 of (b - a), and a 16x finer grid must cut
    # the error by at least 16x (7/5 order predicts about 48x).
    idx = [1, 7, N // 4, N // 2 - 1, N // 2, 3 * N // 4 + 1, N - 1]
    ref = _exact_F_knots(func, params, a, b, N, idx)
    X, X64, flags = O.optimal_knots(func, params, a, b, N)
    err = np.max(np.abs(X64[idx] - ref))
    assert err <= 5e-6 * (b - a)
    Xf, Xf64, _ = O.optimal_knots(func, params, a, b, N, M=4096 * N)
    assert np.max(np.abs(Xf64[idx] - ref)) <= err / 16.0


def test_affine_function_degenerates_to_uniform():
    X, X64, flags = O.optimal_knots(O.POLY, (1.0, -2.0), -1.0, 3.0, 40)
    U, _ = O.uniform_knots(-1.0, 3.0, 40)
    assert flags == O.FLAG_DEGENERATE
    assert np.array_equal(X, U)


def test_knots_strictly_increasing_for_workloads():
    for func, params, a, b in [(O.GAUSSIAN, (1.0, 1.0), -5, 5), (O.LORENTZIAN, (1.0, 1.0), -20, 20),
                               (O.BESSEL_J0, (1.0,), 0, 50)]:
        for N in (16, 256, 4096):
            X, X64, flags = O.optimal_knots(func, params, a, b, N)
            assert flags == 0
            assert np.all(np.diff(X) > 0)
            assert X[0] == a and X[-1] == b


def test_knot_collapse_is_detected():
    # A domain only a few FP32 ulps wide cannot hold 64 distinct FP32 knots.
    a = 1.0
    b = float(np.nextafter(np.nextafter(np.float32(1.0), np.float32(2)), np.float32(2)))
    X, X64, flags = O.optimal_knots(O.GAUSSIAN, (1.0, 1.0), a, b, 64)
    assert flags & O.FLAG_KNOTS_COLLAPSED
    with pytest.raises(O.KnotCollapse):
        O.build_table(O.GAUSSIAN, (1.0, 1.0), a, b, 64, O.UNIFORM, O.INTERP)


def test_invalid_arguments():
    with pytest.raises(ValueError):
        O.build_table(O.GAUSSIAN, None, 1.0, 1.0, 8)
    with pytest.raises(ValueError):
        O.build_table(O.GAUSSIAN, None, 0.0, 1.0, 0)
    with pytest.raises(ValueError):
        O.build_table(O.GAUSSIAN, None, 0.0, float("inf"), 4)


def test_equalised_error_per_segment():
    # Sec. III-B1: on T^(*) every segment carries about the same
    # |f''|_max h^(5/2); check the spread is small for a large N.
    N = 2048
    X, _, _ = O.optimal_knots(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, N)
    h = np.diff(X)
    mid = 0.5 * (X[1:] + X[:-1])
    c = np.abs(O.f_second(O.GAUSSIAN, (1.0, 1.0), mid)) ** 0.4 * h
    # Away from the zeros of f'' (where the density vanishes) the products agree.
    far = np.abs(np.abs(mid) - 1.0) > 0.2
    assert np.max(c[far]) / np.min(c[far]) < 1.02
