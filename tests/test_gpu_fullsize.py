"""Parity at the full workload sizes, in the launch configuration the
benchmark times (library defaults): every 4096th output plus every point
within 1e-5 of a knot is checked against the FP64 oracle's own table; size-
independent properties (finite, within the vertex-value range) are checked on
all outputs on the GPU."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import GRAD_TOL, Y_TOL, device, fmax_abs, library, say

pytestmark = pytest.mark.gpu


def _sample_idx(x, X, stride=4096):
    idx = np.arange(0, len(x), stride)
    # points near knots (the hardest segment decisions)
    pos = np.searchsorted(X, x.astype(np.float64))
    pos = np.clip(pos, 1, len(X) - 1)
    near = np.minimum(np.abs(x - X[pos]), np.abs(x - X[pos - 1])) <= 1e-5
    return np.union1d(idx, np.nonzero(near)[0][:200000])


def _check_forward(P, spec, x_h, label):
    dev = device()
    t = P.pwl_build(spec["func"], spec["params"], spec["a"], spec["b"], spec["N"], spec["partition"],
                    spec["values"])
    x = torch.from_numpy(x_h).to(dev)
    y = P.pwl_eval(t, x)
    d = P.pwl_table_download(t)
    vmin, vmax = float(d["values"].min()), float(d["values"].max())
    assert bool(torch.isfinite(y).all())
    assert float(y.min()) >= vmin - 1e-6 and float(y.max()) <= vmax + 1e-6
    ref = O.build_table(spec["func"], spec["params"], spec["a"], spec["b"], spec["N"], spec["partition"],
                        spec["values"])
    idx = _sample_idx(x_h, ref["X"])
    ys = y[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    yr = O.evaluate(ref["X"], ref["v"], x_h[idx].astype(np.float64))
    err = np.max(np.abs(ys - yr)) / fmax_abs(spec["func"], spec["params"], spec["a"], spec["b"])
    say("  %s: %d points, %d sampled, max err %.3e max|f|" % (label, len(x_h), len(idx), err))
    assert err <= Y_TOL
    t.free()


def test_headline_workload_full_size():
    import paper_1510_02975_amd as P
    library()
    spec = dict(W.GAUSS_BIG)
    _check_forward(P, spec, W.gauss_big_points(spec["n"]), "gauss N=1024 2^28")


@pytest.mark.parametrize("which,N,vals", [("lorentz", 4096, 1), ("j0", 4096, 0), ("j0", 256, 1),
                                          ("lorentz", 1024, 0)])
def test_lorentzian_and_j0_full_size(which, N, vals):
    import paper_1510_02975_amd as P
    library()
    spec = dict(W.LORENTZ if which == "lorentz" else W.BESSEL)
    spec["N"], spec["values"] = N, vals
    x = W.uniform_points(spec["a"], spec["b"], spec["n"], 0)
    _check_forward(P, spec, x, "%s N=%d v=%d 2^27" % (which, N, vals))


def test_gradient_workload_full_size():
    import paper_1510_02975_amd as P
    library()
    dev = device()
    spec = dict(W.GRAD)
    x_h, g_h = W.grad_inputs(spec["n"])
    t = P.pwl_build(spec["func"], spec["params"], spec["a"], spec["b"], spec["N"], spec["partition"],
                    spec["values"])
    y, dx, dv = P.pwl_eval_backward(t, torch.from_numpy(x_h).to(dev), torch.from_numpy(g_h).to(dev))
    d = P.pwl_table_download(t)
    X, v = d["knots"].astype(np.float64), d["values"].astype(np.float64)
    # dL/dv over all 2^26 points (the oracle's bincount is cheap)
    x64, g64 = x_h.astype(np.float64), g_h.astype(np.float64)
    _, _, dvr = O.evaluate_backward(X, v, x64, g64)
    _, _, wk = O.evaluate_backward(X, np.zeros(len(X)), x64, np.abs(g64))
    dvg = dv.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(dvg - dvr) <= GRAD_TOL * wk + 1e-30)
    assert abs(dvg.sum() - g64.sum()) <= 1e-5 * np.abs(g64).sum()
    idx = _sample_idx(x_h, X)
    yr, dxr, _ = O.evaluate_backward(X, v, x64[idx], g64[idx])
    it = torch.from_numpy(idx).to(dev)
    assert np.max(np.abs(y[it].cpu().numpy() - yr)) <= Y_TOL
    i = O.locate(X, x64[idx])
    slope = (v[i + 1] - v[i]) / (X[i + 1] - X[i])
    assert np.all(np.abs(dx[it].cpu().numpy() - dxr) <= GRAD_TOL * np.abs(g64[idx] * slope) + 1e-30)
    say("  gradient workload 2^26: dv max rel %.2e" % np.max(np.abs(dvg - dvr) / np.maximum(wk, 1e-30)))
    t.free()


def test_many_tables_full_size():
    import paper_1510_02975_amd as P
    library()
    dev = device()
    specs = W.many_tables(T=4096, total_points=1 << 28, seed=2)
    tabs = [P.pwl_build(s["func"], s["params"], s["a"], s["b"], s["N"], s["partition"], s["values"],
                        check=False) for s in specs]
    for t in tabs:
        assert P.pwl_table_check(t) == 0
    x_h, offs = W.many_tables_points(specs, seed=0)
    x = torch.from_numpy(x_h).to(dev)
    bt = P.pwl_batch_create(tabs, offs)
    y = P.pwl_batch_eval(bt, x)
    assert bool(torch.isfinite(y).all())
    rng = np.random.default_rng(1)
    worst = 0.0
    for k in rng.choice(len(specs), 48, replace=False):
        s, o0, o1 = specs[k], int(offs[k]), int(offs[k + 1])
        if o1 == o0:
            continue
        ref = O.build_table(s["func"], s["params"], s["a"], s["b"], s["N"], s["partition"], s["values"])
        idx = np.arange(o0, o1, max(1, (o1 - o0) // 2000))
        yr = O.evaluate(ref["X"], ref["v"], x_h[idx].astype(np.float64))
        err = np.max(np.abs(y[torch.from_numpy(idx).to(dev)].cpu().numpy() - yr)) / \
            fmax_abs(s["func"], s["params"], s["a"], s["b"])
        worst = max(worst, err)
    say("  many tables: %d points, worst sampled err %.3e max|f|" % (len(x_h), worst))
    assert worst <= Y_TOL
    bt.free()
    for t in tabs:
        t.free()
