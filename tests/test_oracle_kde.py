"""Pins of the oracle's per-pixel kernel sums (the sample application of
Sec. VI-A) against closed forms and brute force."""

import math

import numpy as np

import oracle as O


def test_history_equal_to_frame_gives_one():
    rng = np.random.default_rng(0)
    f = rng.integers(0, 256, (5, 7, 4), dtype=np.uint8)
    h = np.stack([f] * 3)
    L = O.kde_likelihood(f, h, 0, (5.0, 6.0, 7.0))
    assert np.allclose(L, 1.0, rtol=0, atol=1e-15)


def test_single_sample_closed_form():
    f = np.array([[[10, 200, 30, 255]]], np.uint8)
    h = np.array([[[[20, 190, 33, 0]]]], np.uint8)
    s = (4.0, 5.0, 6.0)
    want = math.exp(-0.5 * ((10 - 20) / 4.0) ** 2) * math.exp(-0.5 * ((200 - 190) / 5.0) ** 2) * \
        math.exp(-0.5 * ((30 - 33) / 6.0) ** 2)
    assert abs(O.kde_likelihood(f, h, 0, s)[0, 0] - want) <= 1e-15
    # a 1 x 1 image: every window position clamps to the one pixel
    assert abs(O.kde_likelihood(f, h, 2, s)[0, 0] - want) <= 1e-15


def test_brute_force_small_image():
    rng = np.random.default_rng(1)
    H, W, T, r = 3, 4, 2, 1
    f = rng.integers(0, 256, (H, W, 4), dtype=np.uint8)
    h = rng.integers(0, 256, (T, H, W, 4), dtype=np.uint8)
    s = (30.0, 40.0, 50.0)
    L = O.kde_likelihood(f, h, r, s)
    for y in range(H):
        for x in range(W):
            acc = 0.0
            for k in range(T):
                for dy in range(-r, r + 1):
                    for dx in range(-r, r + 1):
                        yy, xx = min(max(y + dy, 0), H - 1), min(max(x + dx, 0), W - 1)
                        term = 1.0
                        for c in range(3):
                            u = (float(f[y, x, c]) - float(h[k, yy, xx, c])) / s[c]
                            term *= math.exp(-0.5 * u * u)
                        acc += term
            assert abs(L[y, x] - acc / (T * (2 * r + 1) ** 2)) <= 1e-15
