"""Plain FP64 CPU oracle for continuous piecewise-linear (CPWL) approximation.

Berjon, Gallego, Cuevas, Moran, Garcia, "Optimal Piecewise Linear Function
Approximation for GPU-based Applications", IEEE Trans. Cybernetics 2015
(arXiv 1510.02975).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously correct
reference that the HIP library is checked against.  Only the test suite, the
package smoke check and the CPU-baseline leg of the benchmark may import it;
the library never does, and this module imports nothing from the library.

Everything is float64 NumPy/SciPy, written in the paper's notation:
  partition T : knots a = x_0 < x_1 < ... < x_N = b        (Sec. II-B)
  hat basis   : phi_0 .. phi_N, half hats at the ends      (Sec. II-B)
  pi_T f      : linear interpolant, v_i = f(x_i)            (Sec. II-B1)
  P_T f       : L2 orthogonal projection, M c = b           (Sec. II-B2)
  T^(*)       : quasi-optimal partition F(x_i) = i/N        (Sec. III-B1)
  Algorithm 1 : locate, fractional distance, lerp           (Sec. IV)

Readings of the paper that this oracle fixes (each also listed in the design
notes of the repository):
  * the density is |f''|^(2/5) (the paper writes (f'')^(2/5));
  * F is discretised on M = 256 N equal cells of [a, b] with the trapezoid
    rule; the knot for target tau_i = i S_M / N is found in the first cell j
    whose cumulative sum reaches tau_i and inverted linearly inside it;
  * knots with |x_i| <= 1e-12 (b - a) are snapped to 0, then every knot is
    rounded to FP32; the domain end points a, b are themselves rounded to FP32
    first; all later quantities use the FP32 knots promoted to FP64;
  * f'' identically zero on the grid (affine f) falls back to the uniform
    partition and raises the "degenerate" flag;
  * evaluation clamps x to [a, b]; x = b belongs to segment N-1 with
    fractional distance 1; a point exactly on an interior knot belongs to the
    segment on its right (Algorithm 1 uses x_{i-1} <= x < x_i); NaN x gives
    NaN y and NaN dL/dx and adds nothing to dL/dv.
"""

import collections
import math

import numpy as np
from scipy import special

# Function identifiers (the same numbering the C ABI uses).
GAUSSIAN = 0     # amp * exp(-x^2 / (2 s^2));  params (s, amp)
LORENTZIAN = 1   # amp / (1 + (x / g)^2);      params (g, amp)
BESSEL_J0 = 2    # amp * J0(x);                params (amp,)
POLY = 16        # sum_k c_k x^k, degree <= 5; params (c0, ..., c5)
EXP = 17         # amp * exp(alpha x);         params (alpha, amp)
SAMPLED = 32     # any f given by samples;     params Samples(f, f2, a, b)

# f_i = f(t_i) and f2_i = f''(t_i) at t_i = a + i (b - a) / S, i = 0..S.
# Between samples f is the cubic spline with these values and second
# derivatives (the standard representation of a cubic spline by its moments),
# so f'' is the linear interpolant of f2.
Samples = collections.namedtuple("Samples", "f f2 a b")

UNIFORM, OPTIMAL = 0, 1
INTERP, PROJ = 0, 1

FLAG_DEGENERATE = 1        # f'' == 0 on the grid: uniform fallback
FLAG_KNOTS_COLLAPSED = 2   # FP32 knots not strictly increasing

FINE_CELLS_PER_SEGMENT = 256   # M = 256 N


class KnotCollapse(ValueError):
    """FP32 rounding made two knots equal (or out of order)."""


def _default_params(func, params):
    if func == SAMPLED:
        if not isinstance(params, Samples):
            raise ValueError("a sampled function takes a Samples(f, f2, a, b)")
        return params
    if params is None or len(params) == 0:
        return {GAUSSIAN: (1.0, 1.0), LORENTZIAN: (1.0, 1.0), BESSEL_J0: (1.0,),
                POLY: (0.0,), EXP: (1.0, 1.0)}[func]
    return tuple(float(p) for p in params)


def fl32(x):
    """Round float64 values to the nearest FP32 value and promote back."""
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# The approximated functions and their second derivatives.
# Gaussian (Sec. VI-A), Lorentzian (Sec. VI-B), Bessel J0 (Sec. VI-C); the
# normalisation constants of the paper are folded into `amp`.
# ---------------------------------------------------------------------------

def _sample_cell(smp, x):
    """Interval i (end intervals extended) and local coordinate u of x."""
    S = len(smp.f) - 1
    h = (smp.b - smp.a) / S
    s = (x - smp.a) / h
    i = np.clip(np.floor(s), 0, S - 1).astype(np.int64)
    return i, s - i, h


def _spline_value(smp, x):
    """On [t_i, t_{i+1}] with u = (x - t_i) / h, the cubic whose values are
    f_i, f_{i+1} and whose second derivatives are f2_i, f2_{i+1}:
    (1-u) f_i + u f_{i+1} - h^2 u (1-u) ((2-u) f2_i + (1+u) f2_{i+1}) / 6."""
    f, f2 = np.asarray(smp.f, np.float64), np.asarray(smp.f2, np.float64)
    i, u, h = _sample_cell(smp, x)
    return ((1.0 - u) * f[i] + u * f[i + 1]
            - h * h * u * (1.0 - u) * ((2.0 - u) * f2[i] + (1.0 + u) * f2[i + 1]) / 6.0)


def _spline_second(smp, x):
    f2 = np.asarray(smp.f2, np.float64)
    i, u, _ = _sample_cell(smp, x)
    return (1.0 - u) * f2[i] + u * f2[i + 1]


def f_value(func, params, x):
    p = _default_params(func, params)
    x = np.asarray(x, dtype=np.float64)
    if func == SAMPLED:
        return _spline_value(p, x)
    if func == GAUSSIAN:
        s, amp = p[0], (p[1] if len(p) > 1 else 1.0)
        return amp * np.exp(-(x * x) / (2.0 * s * s))
    if func == LORENTZIAN:
        g, amp = p[0], (p[1] if len(p) > 1 else 1.0)
        u = x / g
        return amp / (1.0 + u * u)
    if func == BESSEL_J0:
        amp = p[0]
        return amp * special.j0(x)
    if func == POLY:
        return np.polynomial.polynomial.polyval(x, np.array(p))
    if func == EXP:
        alpha, amp = p[0], (p[1] if len(p) > 1 else 1.0)
        return amp * np.exp(alpha * x)
    raise ValueError("unknown function id %r" % (func,))


def f_second(func, params, x):
    """f''(x), written from calculus (independent of any finite difference)."""
    p = _default_params(func, params)
    x = np.asarray(x, dtype=np.float64)
    if func == SAMPLED:
        return _spline_second(p, x)
    if func == GAUSSIAN:
        s, amp = p[0], (p[1] if len(p) > 1 else 1.0)
        return amp * ((x * x) / s ** 4 - 1.0 / (s * s)) * np.exp(-(x * x) / (2.0 * s * s))
    if func == LORENTZIAN:
        g, amp = p[0], (p[1] if len(p) > 1 else 1.0)
        u = x / g
        return amp * (6.0 * u * u - 2.0) / (g * g * (1.0 + u * u) ** 3)
    if func == BESSEL_J0:
        amp = p[0]
        # J0' = -J1 and J1' = (J0 - J2)/2, hence J0'' = (J2 - J0)/2.
        return amp * 0.5 * (special.jv(2, x) - special.j0(x))
    if func == POLY:
        c = np.array(p)
        d2 = np.polynomial.polynomial.polyder(c, 2) if len(c) > 2 else np.array([0.0])
        return np.polynomial.polynomial.polyval(x, d2) + 0.0 * x
    if func == EXP:
        alpha, amp = p[0], (p[1] if len(p) > 1 else 1.0)
        return amp * alpha * alpha * np.exp(alpha * x)
    raise ValueError("unknown function id %r" % (func,))


# ---------------------------------------------------------------------------
# Partitions (Sec. II-B and Sec. III-B1).
# ---------------------------------------------------------------------------

def domain32(a, b):
    """The table domain: both end points rounded to FP32."""
    a32, b32 = float(fl32(a)), float(fl32(b))
    if not (math.isfinite(a32) and math.isfinite(b32) and a32 < b32):
        raise ValueError("need finite a < b after rounding to FP32")
    return a32, b32


def uniform_knots(a, b, N):
    """Uniform partition T_U: x_k = a + (b - a) k / N (Sec. IV, uniform case).

    Returns (X32, X64): the FP32 knots promoted to float64, and the float64
    knots before rounding.
    """
    a, b = domain32(a, b)
    k = np.arange(N + 1, dtype=np.float64)
    X64 = a + ((b - a) * k) / N
    X64[0], X64[N] = a, b
    return fl32(X64), X64


def density(func, params, t):
    """Local knot density lkd(x) = |f''(x)|^(2/5) (eq. for lkd, Sec. III-B1)."""
    return np.abs(f_second(func, params, t)) ** 0.4


def cumulative_density(func, params, a, b, M):
    """Grid t_j = a + j dt and trapezoid partial sums S_j of the density.

    S_j approximates the integral of |f''|^(2/5) from a to t_j, i.e. the
    numerator of F(x) (Sec. III-B1); S_M is the normaliser.
    """
    dt = (b - a) / M
    t = a + np.arange(M + 1, dtype=np.float64) * dt
    d = density(func, params, t)
    inc = (d[:-1] + d[1:]) * (dt / 2.0)
    S = np.empty(M + 1)
    S[0] = 0.0
    S[1:] = np.cumsum(inc)
    return t, S, dt


def optimal_knots(func, params, a, b, N, M=None):
    """Quasi-optimal partition T^(*): F(x_i) = i/N (Sec. III-B1).

    Follows the procedure step by step: the range of F is cut into N equal
    sub-ranges and each knot is the abscissa of a cut.  F is the normalised
    cumulative integral of |f''|^(2/5), discretised as described in the module
    header.  Returns (X32, X64, flags).
    """
    a, b = domain32(a, b)
    if M is None:
        M = FINE_CELLS_PER_SEGMENT * N
    t, S, dt = cumulative_density(func, params, a, b, M)
    total = S[M]
    if not (total > 0.0) or not math.isfinite(total):
        X32, X64 = uniform_knots(a, b, N)
        return X32, X64, FLAG_DEGENERATE
    X64 = np.empty(N + 1)
    X64[0], X64[N] = a, b
    snap = 1e-12 * (b - a)
    for i in range(1, N):
        tau = (i * total) / N                       # target value of the cumulative sum
        j = int(np.searchsorted(S, tau, side="left"))   # smallest j with S_j >= tau
        frac = (tau - S[j - 1]) / (S[j] - S[j - 1])
        x = t[j - 1] + frac * dt
        if abs(x) <= snap:
            x = 0.0
        X64[i] = x
    X32 = fl32(X64)
    flags = 0
    if not np.all(np.diff(X32) > 0.0):
        flags |= FLAG_KNOTS_COLLAPSED
    return X32, X64, flags


# ---------------------------------------------------------------------------
# Vertex values: interpolant (Sec. II-B1) and L2 projection (Sec. II-B2).
# ---------------------------------------------------------------------------

def interp_values(func, params, X):
    """pi_T f: nodal values v_i = f(x_i) at the (FP32) knots."""
    return f_value(func, params, np.asarray(X, dtype=np.float64))


def mass_matrix(X):
    """Gram matrix m_ij = <phi_i, phi_j> as three diagonals (lower, diag, upper).

    Assembled from the element matrix (h/6) [[2, 1], [1, 2]] of each segment,
    which is the quadratic form h/3 (d0^2 + d1^2 + d0 d1) of Appendix B; the
    end hats are half hats, so they collect one element only.
    """
    X = np.asarray(X, dtype=np.float64)
    h = np.diff(X)
    N = len(h)
    diag = np.zeros(N + 1)
    diag[:-1] += 2.0 * h / 6.0
    diag[1:] += 2.0 * h / 6.0
    off = h / 6.0
    return off.copy(), diag, off.copy()


_GL_CACHE = {}


def gauss_legendre01(Q):
    """Q-point Gauss-Legendre nodes and weights on [0, 1]."""
    if Q not in _GL_CACHE:
        z, w = np.polynomial.legendre.leggauss(Q)
        _GL_CACHE[Q] = ((z + 1.0) / 2.0, w / 2.0)
    return _GL_CACHE[Q]


def hat_inner_products(func, params, X, Q=16):
    """b_i = <f, phi_i> by Q-point Gauss-Legendre on every segment."""
    X = np.asarray(X, dtype=np.float64)
    N = len(X) - 1
    t, w = gauss_legendre01(Q)
    h = np.diff(X)
    xq = X[:-1, None] + h[:, None] * t[None, :]
    fq = f_value(func, params, xq)
    left = h * np.sum(w * (1.0 - t) * fq, axis=1)   # integral of f * phi_{k} on segment k+1
    right = h * np.sum(w * t * fq, axis=1)          # integral of f * phi_{k+1} on segment k+1
    bvec = np.zeros(N + 1)
    bvec[:-1] += left
    bvec[1:] += right
    return bvec


def thomas(lower, diag, upper, rhs):
    """Thomas algorithm (Gaussian elimination for a tridiagonal system).

    lower[k] = m_{k+1,k}, upper[k] = m_{k,k+1}; no pivoting (the Gram matrix is
    strictly diagonally dominant, Sec. II-B2).
    """
    n = len(diag)
    cp = np.zeros(n)
    dp = np.zeros(n)
    cp[0] = upper[0] / diag[0] if n > 1 else 0.0
    dp[0] = rhs[0] / diag[0]
    for k in range(1, n):
        den = diag[k] - lower[k - 1] * cp[k - 1]
        cp[k] = upper[k] / den if k < n - 1 else 0.0
        dp[k] = (rhs[k] - lower[k - 1] * dp[k - 1]) / den
    x = np.zeros(n)
    x[n - 1] = dp[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = dp[k] - cp[k] * x[k + 1]
    return x


def proj_values(func, params, X, Q=16):
    """P_T f: coefficients c solving M c = b (Sec. II-B2)."""
    lo, di, up = mass_matrix(X)
    return thomas(lo, di, up, hat_inner_products(func, params, X, Q))


# ---------------------------------------------------------------------------
# Table construction.
# ---------------------------------------------------------------------------

def build_table(func, params, a, b, N, partition=OPTIMAL, values=PROJ, M=None):
    """Knots and vertex values of one CPWL table.

    Returns a dict with X (FP32 knots as float64), X64 (knots before FP32
    rounding), v (float64 vertex values), flags, a, b, N.
    Raises KnotCollapse if the FP32 knots are not strictly increasing.
    """
    N = int(N)
    if N < 1:
        raise ValueError("N must be >= 1")
    a, b = domain32(a, b)
    if partition == UNIFORM:
        X, X64 = uniform_knots(a, b, N)
        flags = 0 if np.all(np.diff(X) > 0.0) else FLAG_KNOTS_COLLAPSED
    elif partition == OPTIMAL:
        X, X64, flags = optimal_knots(func, params, a, b, N, M)
    else:
        raise ValueError("unknown partition %r" % (partition,))
    if flags & FLAG_KNOTS_COLLAPSED:
        raise KnotCollapse("FP32 knots are not strictly increasing")
    if values == INTERP:
        v = interp_values(func, params, X)
    elif values == PROJ:
        v = proj_values(func, params, X)
    else:
        raise ValueError("unknown values kind %r" % (values,))
    return {"X": X, "X64": X64, "v": v, "flags": flags, "a": a, "b": b, "N": N,
            "func": func, "params": _default_params(func, params),
            "partition": partition, "values": values}


# ---------------------------------------------------------------------------
# Algorithm 1 (Sec. IV): CPWL evaluation, and its exact derivative.
# ---------------------------------------------------------------------------

def locate(X, x):
    """Segment index i (0-based) with X[i] <= x < X[i+1], clamped to [0, N-1].

    x is clamped to [X[0], X[N]] first; x = X[N] maps to N-1.
    """
    X = np.asarray(X, dtype=np.float64)
    N = len(X) - 1
    xc = np.clip(np.asarray(x, dtype=np.float64), X[0], X[N])
    i = np.searchsorted(X, xc, side="right") - 1
    return np.clip(i, 0, N - 1)


def evaluate(X, v, x):
    """v(x*) = (1 - delta) v(x_{i-1}) + delta v(x_i) (Algorithm 1)."""
    X = np.asarray(X, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    N = len(X) - 1
    xc = np.clip(x, X[0], X[N])
    i = locate(X, xc)
    delta = (xc - X[i]) / (X[i + 1] - X[i])
    return (1.0 - delta) * v[i] + delta * v[i + 1]


def evaluate_backward(X, v, x, g):
    """Exact derivative of Algorithm 1 for an upstream gradient g.

    Returns (y, dL/dx, dL/dv).  dL/dx = g * slope inside [a, b] (left slope at
    x = b), 0 outside; dL/dv_i += (1 - delta) g, dL/dv_{i+1} += delta g.
    """
    X = np.asarray(X, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    N = len(X) - 1
    xc = np.clip(x, X[0], X[N])
    i = locate(X, xc)
    h = X[i + 1] - X[i]
    delta = (xc - X[i]) / h
    y = (1.0 - delta) * v[i] + delta * v[i + 1]
    slope = (v[i + 1] - v[i]) / h
    inside = (x >= X[0]) & (x <= X[N])
    dx = np.where(inside, g * slope, 0.0)
    nan = np.isnan(x)
    dx = np.where(nan, np.nan, dx)
    ok = ~nan
    dv = (np.bincount(i[ok], weights=((1.0 - delta) * g)[ok], minlength=N + 1)
          + np.bincount(i[ok] + 1, weights=(delta * g)[ok], minlength=N + 1))
    return y, dx, dv


# ---------------------------------------------------------------------------
# Approximation errors and the paper's predicted values (Sec. III).
# ---------------------------------------------------------------------------

def l2_error(func, params, X, v, Q=16):
    """||f - v||_{L2[a,b]} by Q-point Gauss-Legendre on each segment."""
    X = np.asarray(X, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    t, w = gauss_legendre01(Q)
    h = np.diff(X)
    xq = X[:-1, None] + h[:, None] * t[None, :]
    line = v[:-1, None] * (1.0 - t[None, :]) + v[1:, None] * t[None, :]
    err2 = (f_value(func, params, xq) - line) ** 2
    return math.sqrt(float(np.sum(h * np.sum(w * err2, axis=1))))


def linf_error(func, params, X, v, samples=33, refine_iters=60):
    """max |f - v| on [a, b]: 33 samples per segment, then golden-section
    refinement around the best sample of the worst segments."""
    X = np.asarray(X, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    h = np.diff(X)
    s = np.linspace(0.0, 1.0, samples)
    xs = X[:-1, None] + h[:, None] * s[None, :]
    line = v[:-1, None] * (1.0 - s[None, :]) + v[1:, None] * s[None, :]
    e = np.abs(f_value(func, params, xs) - line)
    best = float(e.max())
    seg_max = e.max(axis=1)
    order = np.argsort(seg_max)[::-1][:8]
    gr = (math.sqrt(5.0) - 1.0) / 2.0
    for k in order:
        j = int(np.argmax(e[k]))
        lo = max(j - 1, 0) / (samples - 1)
        hi = min(j + 1, samples - 1) / (samples - 1)

        def err(tt, k=k):
            xx = X[k] + h[k] * tt
            return abs(float(f_value(func, params, xx)) - (v[k] * (1.0 - tt) + v[k + 1] * tt))
        c, d = hi - gr * (hi - lo), lo + gr * (hi - lo)
        fc, fd = err(c), err(d)
        for _ in range(refine_iters):
            if fc > fd:
                hi, d, fd = d, c, fc
                c = hi - gr * (hi - lo)
                fc = err(c)
            else:
                lo, c, fc = c, d, fd
                d = lo + gr * (hi - lo)
                fd = err(d)
        best = max(best, fc, fd)
    return best


def second_derivative_zeros(func, params, a, b, grid=20001):
    """Zeros of f'' in (a, b): sign changes on a fine grid refined by brentq."""
    from scipy.optimize import brentq
    t = np.linspace(a, b, grid)
    s = f_second(func, params, t)
    zs = []
    for k in range(grid - 1):
        if s[k] == 0.0 and a < t[k] < b:
            zs.append(float(t[k]))
        elif s[k] * s[k + 1] < 0.0:
            zs.append(brentq(lambda z: float(f_second(func, params, z)), t[k], t[k + 1],
                             xtol=1e-15, rtol=1e-15))
    return sorted(set(zs))


def density_integral(func, params, a, b):
    """Integral of |f''|^(2/5) over [a, b] by adaptive quadrature with
    break points at the zeros of f''."""
    from scipy.integrate import quad
    pts = [a] + second_derivative_zeros(func, params, a, b) + [b]
    tot = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        val, _ = quad(lambda z: float(density(func, params, z)), lo, hi,
                      limit=400, epsabs=0.0, epsrel=1e-12)
        tot += val
    return tot


def second_derivative_norms(func, params, a, b):
    """(||f''||_{L2[a,b]}, max |f''| on [a, b])."""
    from scipy.integrate import quad
    from scipy.optimize import minimize_scalar
    pts = [a] + second_derivative_zeros(func, params, a, b) + [b]
    sq = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        val, _ = quad(lambda z: float(f_second(func, params, z)) ** 2, lo, hi,
                      limit=400, epsabs=0.0, epsrel=1e-12)
        sq += val
    t = np.linspace(a, b, 200001)
    m = np.abs(f_second(func, params, t))
    k = int(np.argmax(m))
    lo, hi = t[max(k - 1, 0)], t[min(k + 1, len(t) - 1)]
    r = minimize_scalar(lambda z: -abs(float(f_second(func, params, z))),
                        bounds=(lo, hi), method="bounded", options={"xatol": 1e-14})
    return math.sqrt(sq), max(float(m[k]), -float(r.fun))


def predicted_errors(func, params, a, b, N):
    """The paper's error predictions and the derived L-infinity ones.

    L2 (Sec. III-B2):
      Result 4  interp on T^(*):  (int |f''|^(2/5))^(5/2) / (N^2 sqrt(120))
      Result 5  proj on T^(*):    Result 4 / sqrt(6)
      Result 6  interp on T_U:    (b - a)^2 ||f''|| / (N^2 sqrt(120))
      proj on T_U:                Result 6 / sqrt(6) (per-interval Result 3)
    L-inf (from eq. (interpolant-difference) and the minimisers of Appendix B,
    with f'' frozen per segment): h^2 |f''| / 8 (interp), h^2 |f''| / 12 (proj).
    """
    a, b = domain32(a, b)
    I25 = density_integral(func, params, a, b)
    l2f2, maxf2 = second_derivative_norms(func, params, a, b)
    r120 = math.sqrt(120.0)
    r6 = math.sqrt(6.0)
    out = {
        "l2": {
            (OPTIMAL, INTERP): I25 ** 2.5 / (N * N * r120),
            (OPTIMAL, PROJ): I25 ** 2.5 / (N * N * r120) / r6,
            (UNIFORM, INTERP): (b - a) ** 2 * l2f2 / (N * N * r120),
            (UNIFORM, PROJ): (b - a) ** 2 * l2f2 / (N * N * r120) / r6,
        },
        "linf": {
            (OPTIMAL, INTERP): maxf2 ** 0.2 * I25 ** 2 / (8.0 * N * N),
            (OPTIMAL, PROJ): maxf2 ** 0.2 * I25 ** 2 / (12.0 * N * N),
            (UNIFORM, INTERP): (b - a) ** 2 * maxf2 / (8.0 * N * N),
            (UNIFORM, PROJ): (b - a) ** 2 * maxf2 / (12.0 * N * N),
        },
        "density_integral": I25,
        "f2_l2": l2f2,
        "f2_max": maxf2,
    }
    return out


def result1_bound(func, params, X, grid_per_segment=65):
    """Rigorous Result 1: sqrt(sum_i (max_{I_i} |f''|)^2 h_i^5 / 120), with the
    per-segment maximum taken on a dense sample plus the end points."""
    X = np.asarray(X, dtype=np.float64)
    h = np.diff(X)
    s = np.linspace(0.0, 1.0, grid_per_segment)
    xs = X[:-1, None] + h[:, None] * s[None, :]
    m = np.abs(f_second(func, params, xs)).max(axis=1)
    return math.sqrt(float(np.sum(m * m * h ** 5 / 120.0)))


# ---------------------------------------------------------------------------
# Sample application (Sec. VI-A): per-pixel sums of Gaussian kernels of a
# nonparametric background model.
# ---------------------------------------------------------------------------

def kde_likelihood(frame, hist, radius, sigma, g=None):
    """For every pixel (y, x) of frame [H, W, >=3] the mean, over the T
    reference frames hist [T, H, W, >=3] and the (2r+1) x (2r+1) window of
    (y, x) (indices clamped to the image), of prod_c g((frame[y, x, c] -
    hist[k, y', x', c]) / sigma[c]) over the first three channels, with
    g(u) = exp(-u^2 / 2) unless another g is given."""
    if g is None:
        def g(u):
            return np.exp(-0.5 * u * u)
    f = np.asarray(frame)[..., :3].astype(np.float64)
    h = np.asarray(hist)[..., :3].astype(np.float64)
    T, H, W = h.shape[:3]
    ys, xs = np.arange(H), np.arange(W)
    acc = np.zeros((H, W))
    for k in range(T):
        for dy in range(-radius, radius + 1):
            yy = np.clip(ys + dy, 0, H - 1)
            for dx in range(-radius, radius + 1):
                xx = np.clip(xs + dx, 0, W - 1)
                hk = h[k][yy][:, xx]
                term = np.ones((H, W))
                for c in range(3):
                    term = term * g((f[..., c] - hk[..., c]) / float(sigma[c]))
                acc += term
    return acc / (T * (2 * radius + 1) ** 2)
