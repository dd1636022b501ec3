"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the
benchmark.

This module only draws random numbers and lays out workload descriptions; it
holds none of the approximation method's arithmetic, and it imports neither
the oracle nor the library.

Recipe (every generator is numpy's PCG64 `default_rng(seed)`, drawn in
float64 and rounded once to float32):
  * gauss_small  Gaussian on [-4, 4], uniform N=64: x = -4 + 8 U, seed 0
  * gauss_big    Gaussian on [-5, 5], optimal N=1024: x = clip(fl32(1.5 Z), -5, 5), seed 0
  * lorentz/j0   uniform x on [-20, 20] / [0, 50], seed 0
  * grad         x ~ N(0, 1) with seed 0, upstream g ~ N(0, 1) with seed 1
  * many tables  seed 2 draws the table parameters; the points of table t
                 continue one seed-0 stream in table order
"""

import math

import numpy as np

GAUSSIAN, LORENTZIAN, BESSEL_J0 = 0, 1, 2
UNIFORM, OPTIMAL = 0, 1
INTERP, PROJ = 0, 1

_CHUNK = 1 << 24


def _chunked(n, draw):
    out = np.empty(n, dtype=np.float32)
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        out[s:e] = draw(e - s)
    return out


def uniform_points(a, b, n, seed=0):
    """n FP32 points fl32(a + (b - a) U), U ~ U[0, 1)."""
    rng = np.random.default_rng(seed)
    return _chunked(int(n), lambda m: (a + (b - a) * rng.random(m)).astype(np.float32))


def normal_points(n, sigma=1.0, seed=0, lo=None, hi=None):
    """n FP32 points fl32(sigma Z), optionally clipped to [lo, hi] after rounding."""
    rng = np.random.default_rng(seed)

    def draw(m):
        x = (sigma * rng.standard_normal(m)).astype(np.float32)
        if lo is not None:
            np.clip(x, np.float32(lo), np.float32(hi), out=x)
        return x
    return _chunked(int(n), draw)


def upstream_grad(n, seed=1):
    """Upstream gradient g ~ N(0, 1) in FP32."""
    return normal_points(n, 1.0, seed)


# --- the named workloads --------------------------------------------------

GAUSS_SMALL = dict(name="gauss_uniform_n64", func=GAUSSIAN, params=(1.0, 1.0), a=-4.0, b=4.0,
                   N=64, partition=UNIFORM, n=1 << 20)
GAUSS_BIG = dict(name="gauss_optimal_n1024_proj", func=GAUSSIAN, params=(1.0, 1.0), a=-5.0,
                 b=5.0, N=1024, partition=OPTIMAL, values=PROJ, n=1 << 28)
LORENTZ = dict(name="lorentz_optimal", func=LORENTZIAN, params=(1.0, 1.0), a=-20.0, b=20.0,
               partition=OPTIMAL, n=1 << 27)
BESSEL = dict(name="j0_optimal", func=BESSEL_J0, params=(1.0,), a=0.0, b=50.0,
              partition=OPTIMAL, n=1 << 27)
GRAD = dict(name="gauss_optimal_n512_proj_fwd_bwd", func=GAUSSIAN, params=(1.0, 1.0), a=-5.0,
            b=5.0, N=512, partition=OPTIMAL, values=PROJ, n=1 << 26)


def gauss_small_points(n=1 << 20, seed=0):
    return uniform_points(-4.0, 4.0, n, seed)


def gauss_big_points(n=1 << 28, seed=0):
    return normal_points(n, 1.5, seed, -5.0, 5.0)


def grad_inputs(n=1 << 26, seed_x=0, seed_g=1):
    return normal_points(n, 1.0, seed_x), upstream_grad(n, seed_g)


def many_tables(T=4096, total_points=1 << 28, seed=2, scale_to_total=True):
    """Descriptions of T tables of uneven size and uneven point counts.

    f is uniform over {Gaussian, Lorentzian, J0}; sigma and gamma are
    log-uniform in [0.1, 10] with domains [-5 sigma, 5 sigma] and
    [-20 gamma, 20 gamma] (end points rounded to FP32), J0 lives on [0, 50];
    N = round(log-uniform[16, 4096]); partition and values kinds are each a
    fair coin; point counts are log-uniform in [2^10, 2^20].  With
    scale_to_total the counts are rescaled to sum to about total_points
    (floor, at least 1), because the raw draw averages about 2^29.2.
    """
    rng = np.random.default_rng(seed)
    kinds = rng.integers(0, 3, T)
    widths = np.exp(rng.uniform(math.log(0.1), math.log(10.0), T))
    Ns = np.rint(np.exp(rng.uniform(math.log(16.0), math.log(4096.0), T))).astype(np.int64)
    parts = rng.integers(0, 2, T)
    vals = rng.integers(0, 2, T)
    counts = np.exp(rng.uniform(math.log(2.0 ** 10), math.log(2.0 ** 20), T))
    if scale_to_total:
        counts = np.maximum(np.floor(counts * (total_points / counts.sum())), 1.0)
    counts = counts.astype(np.int64)
    tables = []
    for t in range(T):
        k = int(kinds[t])
        w = float(widths[t])
        if k == GAUSSIAN:
            params, a, b = (w, 1.0), float(np.float32(-5.0 * w)), float(np.float32(5.0 * w))
        elif k == LORENTZIAN:
            params, a, b = (w, 1.0), float(np.float32(-20.0 * w)), float(np.float32(20.0 * w))
        else:
            params, a, b = (1.0,), 0.0, 50.0
        tables.append(dict(func=k, params=params, a=a, b=b, N=int(Ns[t]),
                           partition=int(parts[t]), values=int(vals[t]), n=int(counts[t])))
    return tables


def many_tables_points(tables, seed=0):
    """Concatenated FP32 points, table by table, uniform on each domain, drawn
    from one seed-`seed` stream; also returns the [T+1] offsets."""
    rng = np.random.default_rng(seed)
    offs = np.zeros(len(tables) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([t["n"] for t in tables])
    x = np.empty(int(offs[-1]), dtype=np.float32)
    for i, t in enumerate(tables):
        m = t["n"]
        x[offs[i]:offs[i + 1]] = (t["a"] + (t["b"] - t["a"]) * rng.random(m)).astype(np.float32)
    return x, offs


# --- sample application: per-pixel sums of Gaussian kernels ----------------
# Nonparametric background model (Sec. VI-A): every pixel of the current
# frame is compared with the pixels of a (2r+1) x (2r+1) window in each of T
# reference frames.  Synthetic scene: a smooth colour field that drifts and
# flickers from frame to frame, plus sensor noise, and a moving square
# "foreground" object in the current frame.  RGBA8, alpha 255.
KDE_CIF = dict(name="kde_cif", H=288, W=352, T=16, radius=2, sigma=(6.0, 6.0, 6.0))


def kde_frames(H, W, T, seed=3):
    """(frame [H, W, 4] uint8, history [T, H, W, 4] uint8)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64), indexing="ij")
    phase = rng.uniform(0.0, 2.0 * math.pi, 3)

    def scene(shift, gain):
        out = np.empty((H, W, 4), dtype=np.float64)
        for c in range(3):
            out[..., c] = 128.0 + 60.0 * np.sin(0.02 * (xx + shift) + 0.03 * yy + phase[c]) * gain
        out[..., 3] = 255.0
        return out

    hist = np.empty((T, H, W, 4), dtype=np.uint8)
    for t in range(T):
        f = scene(0.7 * t, 1.0 + 0.02 * rng.standard_normal())
        f[..., :3] += 4.0 * rng.standard_normal((H, W, 3))
        hist[t] = np.clip(np.rint(f), 0, 255).astype(np.uint8)
    cur = scene(0.7 * T, 1.0)
    cur[..., :3] += 4.0 * rng.standard_normal((H, W, 3))
    s = max(4, min(H, W) // 6)
    y0, x0 = H // 3, W // 2
    cur[y0:y0 + s, x0:x0 + s, :3] = rng.uniform(0.0, 255.0, 3)   # the foreground square
    frame = np.clip(np.rint(cur), 0, 255).astype(np.uint8)
    return frame, hist
