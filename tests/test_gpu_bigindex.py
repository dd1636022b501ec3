"""Point counts past 2^31: every streaming kernel indexes points with 64-bit
integers, and this checks it on 2^31 + 13 points, forward and fused backward,
single-table and batched, in the library's default launch configuration.

The inputs repeat a pattern of P points (P odd, so the 16-byte vectors fall
across the period boundaries at every phase), so the outputs can be checked
in full without running the oracle on 2^31 points: evaluation is pointwise,
so y, dL/dx and the segment indices must repeat bit for bit with the input,
and their first period must match the FP64 oracle; dL/dv, a sum over the
points, must equal the oracle's dL/dv of the pattern times the number of
whole periods plus that of the partial last period."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import GRAD_TOL, Y_TOL, device, fmax_abs, library, say

pytestmark = pytest.mark.gpu

P_LEN = (1 << 20) + 7          # period of the inputs (odd)
N_POINTS = (1 << 31) + 13      # past the largest int32


def _periodic(pat, n):
    """pat repeated to n elements, on the device (a contiguous prefix)."""
    reps = -(-n // pat.numel())
    return pat.repeat(reps)[:n]


def _assert_periodic(t, p):
    """t[i] == t[i mod p] for every i, bit for bit."""
    n = t.numel()
    whole = n // p
    head = t[:p]
    assert torch.equal(t[:whole * p].view(whole, p), head.expand(whole, p))
    assert torch.equal(t[whole * p:], head[:n - whole * p])


def _dv_expected(X, v, x64, g64, n):
    """dL/dv and its normwise scale (sum |g| phi_k) over n points that
    repeat the pattern (x64, g64): whole periods plus the partial one."""
    p = len(x64)
    whole, rem = divmod(n, p)
    _, _, dv = O.evaluate_backward(X, v, x64, g64)
    _, _, wk = O.evaluate_backward(X, np.zeros(len(X)), x64, np.abs(g64))
    _, _, dv_r = O.evaluate_backward(X, v, x64[:rem], g64[:rem])
    _, _, wk_r = O.evaluate_backward(X, np.zeros(len(X)), x64[:rem], np.abs(g64[:rem]))
    return whole * dv + dv_r, whole * wk + wk_r


def _check_first_period(t, spec, x_h, g_h, y, dx, label):
    """First period of y (against the oracle's own table) and dL/dx (on the
    GPU table's knots and values) within the parity tolerances."""
    ref = O.build_table(spec["func"], spec["params"], spec["a"], spec["b"], spec["N"], spec["partition"],
                        spec["values"])
    x64, g64 = x_h.astype(np.float64), g_h.astype(np.float64)
    scale = fmax_abs(spec["func"], spec["params"], spec["a"], spec["b"])
    yerr = np.max(np.abs(y[:len(x_h)].cpu().numpy() - O.evaluate(ref["X"], ref["v"], x64))) / scale
    assert yerr <= Y_TOL
    d = P_mod().pwl_table_download(t)
    X, v = d["knots"].astype(np.float64), d["values"].astype(np.float64)
    if dx is not None:
        _, dxr, _ = O.evaluate_backward(X, v, x64, g64)
        i = O.locate(X, x64)
        slope = (v[i + 1] - v[i]) / (X[i + 1] - X[i])
        dxg = dx[:len(x_h)].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(dxg - dxr) <= GRAD_TOL * np.abs(g64 * slope) + 1e-30)
    say("  %s: first period max err %.3e max|f|" % (label, yerr))
    return X, v


def P_mod():
    import paper_1510_02975_amd as P
    return P


def _build(spec):
    return P_mod().pwl_build(spec["func"], spec["params"], spec["a"], spec["b"], spec["N"], spec["partition"],
                             spec["values"])


def test_single_table_past_int32():
    P = P_mod()
    library()
    dev = device()
    spec = dict(W.GAUSS_BIG)
    x_h = W.gauss_big_points(P_LEN, seed=5)
    g_h = W.upstream_grad(P_LEN, 6)
    say("  single table: %d points, period %d" % (N_POINTS, P_LEN))
    x = _periodic(torch.from_numpy(x_h).to(dev), N_POINTS)
    t = _build(spec)
    y = P.pwl_eval(t, x)
    _assert_periodic(y, P_LEN)
    X, v = _check_first_period(t, spec, x_h, g_h, y, None, "forward")
    del y
    seg = P.pwl_locate(t, x)
    _assert_periodic(seg, P_LEN)
    assert np.array_equal(seg[:P_LEN].cpu().numpy(), O.locate(X, x_h.astype(np.float64)))
    del seg
    g = _periodic(torch.from_numpy(g_h).to(dev), N_POINTS)
    yb, dx, dv = P.pwl_eval_backward(t, x, g)
    _assert_periodic(yb, P_LEN)
    _assert_periodic(dx, P_LEN)
    _check_first_period(t, spec, x_h, g_h, yb, dx, "fused backward")
    dvr, wk = _dv_expected(X, v, x_h.astype(np.float64), g_h.astype(np.float64), N_POINTS)
    dvg = dv.cpu().numpy().astype(np.float64)
    rel = float(np.max(np.abs(dvg - dvr) / np.maximum(wk, 1e-30)))
    say("  fused backward: dL/dv max rel %.2e" % rel)
    assert np.all(np.abs(dvg - dvr) <= GRAD_TOL * wk + 1e-30)
    t.free()


def test_batch_past_int32():
    """Two tables, the first owning 1024 whole periods (2^30 + 7168 points),
    the second the rest (so every table starts a period)."""
    P = P_mod()
    library()
    dev = device()
    specs = [dict(W.GAUSS_BIG), dict(W.LORENTZ, N=700, values=O.INTERP)]
    x_h = W.gauss_big_points(P_LEN, seed=7)
    g_h = W.upstream_grad(P_LEN, 8)
    offs = [0, 1024 * P_LEN, N_POINTS]
    say("  batch: %d points in two tables, period %d" % (N_POINTS, P_LEN))
    tabs = [_build(s) for s in specs]
    x = _periodic(torch.from_numpy(x_h).to(dev), N_POINTS)
    g = _periodic(torch.from_numpy(g_h).to(dev), N_POINTS)
    bt = P.pwl_batch_create(tabs, offs)
    yb, dx, dv = P.pwl_batch_eval_backward(bt, x, g)
    y = P.pwl_batch_eval(bt, x)
    assert torch.equal(y, yb)
    del yb
    dv_h = dv.cpu().numpy().astype(np.float64)
    for k, s in enumerate(specs):
        o0, o1 = offs[k], offs[k + 1]
        _assert_periodic(y[o0:o1], P_LEN)
        _assert_periodic(dx[o0:o1], P_LEN)
        X, v = _check_first_period(tabs[k], s, x_h, g_h, y[o0:o1], dx[o0:o1], "table %d" % k)
        dvr, wk = _dv_expected(X, v, x_h.astype(np.float64), g_h.astype(np.float64), o1 - o0)
        d0, d1 = bt.dv_offsets[k], bt.dv_offsets[k + 1]
        rel = float(np.max(np.abs(dv_h[d0:d1] - dvr) / np.maximum(wk, 1e-30)))
        say("  table %d: dL/dv max rel %.2e" % (k, rel))
        assert np.all(np.abs(dv_h[d0:d1] - dvr) <= GRAD_TOL * wk + 1e-30)
    bt.free()
    for t in tabs:
        t.free()
