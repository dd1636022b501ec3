"""Uniform-partition tables (Sec. IV's equal segments, located through the
index map with K = 2N cells) on domains where FP32 rounding of the knots
and of x - a shifts points across segment ends - far from 0, tiny,
asymmetric, N = 1 and 2 - at every knot and its FP32 neighbours: the
forward equals the binary-search locate bit for bit, the segments equal the
oracle's on the FP32 knots, and the fused backward matches the FP64 oracle
on the downloaded table (a direct index, floor((x - a) N / (b - a)) with a
compare-fix, measured slower than the branch-free map on gfx950)."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import GRAD_TOL, Y_TOL, device, fmax_abs, library, locate_mode, say

pytestmark = pytest.mark.gpu

TABLES = [
    (O.GAUSSIAN, (1.0, 1.0), -4.0, 4.0, 64),
    (O.POLY, (0.0, 0.0, 0.5), 1000.0, 1001.3, 4096),         # knots 5 ulp apart, far from 0
    (O.POLY, (1.0, -2.0, 0.25), -1e-3, 3e-3, 777),           # tiny domain around 0
    (O.LORENTZIAN, (1.0, 1.0), -7.3, 11.9, 1000),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 4096),
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 1),
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 2),
]


def _points(X, a, b, seed):
    pts = [W.uniform_points(a - 0.1 * (b - a), b + 0.1 * (b - a), 100003, seed),
           X, np.nextafter(X, np.float32(-np.inf)), np.nextafter(X, np.float32(np.inf)),
           np.array([a, b, -np.inf, np.inf, np.nan, 0.0, -0.0], np.float32)]
    return np.concatenate(pts).astype(np.float32)


@pytest.mark.parametrize("spec", TABLES, ids=["%s-[%g,%g]-N%d" % (s[0], s[2], s[3], s[4]) for s in TABLES])
@pytest.mark.parametrize("vals", [O.INTERP, O.PROJ])
def test_uniform_tables_at_segment_ends(spec, vals):
    import paper_1510_02975_amd as P
    library()
    dev = device()
    func, p, a, b, N = spec
    t = P.pwl_build(func, p, a, b, N, O.UNIFORM, vals)
    d = P.pwl_table_download(t)
    X = d["knots"]
    x_h = _points(X, np.float32(a), np.float32(b), 11)
    x = torch.from_numpy(x_h).to(dev)
    with locate_mode(P, P.LOCATE_MAP):
        y = P.pwl_eval(t, x).cpu().numpy()
        y_odd = P.pwl_eval(t, x[1:5001]).cpu().numpy()      # scalar (misaligned) path
    with locate_mode(P, P.LOCATE_SEARCH):
        y_bs = P.pwl_eval(t, x).cpu().numpy()
    assert np.array_equal(y, y_bs, equal_nan=True)
    assert np.array_equal(y[1:5001], y_odd, equal_nan=True)
    # segments: the index map's, and the oracle's on the FP32 knots
    seg = P.pwl_locate(t, x).cpu().numpy()
    X64 = X.astype(np.float64)
    ok = ~np.isnan(x_h)
    ref_seg = O.locate(X64, np.clip(x_h[ok].astype(np.float64), X64[0], X64[-1]))
    assert np.array_equal(seg[ok], ref_seg)
    # fused backward on the same points against the oracle (tier ii)
    g_h = W.upstream_grad(len(x_h), 12)
    g = torch.from_numpy(g_h).to(dev)
    yb, dxb, dvb = P.pwl_eval_backward(t, x, g)
    yb, dxb, dvb = yb.cpu().numpy(), dxb.cpu().numpy(), dvb.cpu().numpy()
    assert np.array_equal(yb, y, equal_nan=True)
    v64 = d["values"].astype(np.float64)
    xf, gf = x_h[ok].astype(np.float64), g_h[ok].astype(np.float64)
    yr, dxr, dvr = O.evaluate_backward(X64, v64, xf, gf)
    fmax = max(fmax_abs(func, p, a, b), 1e-30)
    assert np.max(np.abs(yb[ok] - yr)) <= Y_TOL * fmax
    slope = np.abs(np.where(gf != 0.0, dxr / np.where(gf != 0.0, gf, 1.0), 0.0))
    assert np.all(np.abs(dxb[ok] - dxr) <= GRAD_TOL * np.abs(gf) * slope + 1e-30)
    _, _, wk = O.evaluate_backward(X64, np.zeros_like(v64), xf, np.abs(gf))
    assert np.all(np.abs(dvb - dvr) <= GRAD_TOL * wk + 1e-30)
    say("  f=%d [%g, %g] N=%d vals=%d: %d points, segments and outputs match" % (func, a, b, N, vals, len(x_h)))
    t.free()


def test_uniform_batch_matches_single_table():
    """Uniform tables on those domains inside a batch (with one optimal
    table): the batched forward and fused backward equal the per-table
    launches bit for bit."""
    import paper_1510_02975_amd as P
    library()
    dev = device()
    tabs = [P.pwl_build(f, p, a, b, N, O.UNIFORM, O.PROJ) for f, p, a, b, N in TABLES[:5]]
    tabs.append(P.pwl_build(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 300, O.OPTIMAL, O.INTERP))
    xs = [_points(P.pwl_table_download(t)["knots"], np.float32(t.a), np.float32(t.b), 20 + k)
          for k, t in enumerate(tabs)]
    offs = np.concatenate([[0], np.cumsum([len(v) for v in xs])]).astype(np.int64)
    x = torch.from_numpy(np.concatenate(xs)).to(dev)
    g = torch.from_numpy(W.upstream_grad(x.numel(), 21)).to(dev)
    bt = P.pwl_batch_create(tabs, offs)
    y = P.pwl_batch_eval(bt, x)
    yb, dxb, _ = P.pwl_batch_eval_backward(bt, x, g)
    for k, t in enumerate(tabs):
        o0, o1 = int(offs[k]), int(offs[k + 1])
        assert torch.equal(y[o0:o1].isnan(), P.pwl_eval(t, x[o0:o1]).isnan())
        assert torch.equal(torch.nan_to_num(y[o0:o1]), torch.nan_to_num(P.pwl_eval(t, x[o0:o1]))), k
        y1, dx1, _ = P.pwl_eval_backward(t, x[o0:o1], g[o0:o1])
        assert torch.equal(torch.nan_to_num(yb[o0:o1]), torch.nan_to_num(y1)), k
        assert torch.equal(torch.nan_to_num(dxb[o0:o1]), torch.nan_to_num(dx1)), k
    bt.free()
    for t in tabs:
        t.free()
