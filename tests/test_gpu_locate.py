"""The paper's own GPU locate - a branch-free binary search over the knots
(Sec. IV-V), here over the knots staged in LDS - and the default index map,
each against the FP64 oracle: both must return the oracle's segment index
(the segment locate of Algorithm 1) on the GPU's own knots, exactly, and pwl_eval through
either must match the oracle's evaluation; the two modes' outputs are then
bit-identical.  The same for the three arrangements of the per-segment
data in LDS (packed records, structure of arrays, value/slope pairs;
Sec. V), under both locate modes.  Points: random, every knot and its FP32 neighbours, the domain ends,
points outside, +-inf and NaN."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import Y_TOL, device, fmax_abs, library, locate_mode, records_layout, say

pytestmark = pytest.mark.gpu

TABLES = [
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 1024, O.OPTIMAL, O.PROJ),
    (O.GAUSSIAN, (1.0, 1.0), -4.0, 4.0, 64, O.UNIFORM, O.INTERP),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 4096, O.OPTIMAL, O.INTERP),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 777, O.OPTIMAL, O.PROJ),
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 1, O.UNIFORM, O.PROJ),
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 2, O.OPTIMAL, O.INTERP),
    (O.EXP, (1.0, 1.0), 0.0, 3.0, 3, O.OPTIMAL, O.PROJ),
]


def _points(t, a, b):
    """Random points on a widened domain, every knot and its FP32
    neighbours, the ends, +-inf, NaN and signed zeros."""
    import paper_1510_02975_amd as P
    X = P.pwl_table_download(t)["knots"]
    pts = [W.uniform_points(a - 1.0, b + 1.0, 100003, 3),
           X, np.nextafter(X, np.float32(-np.inf)), np.nextafter(X, np.float32(np.inf)),
           np.array([a, b, -np.inf, np.inf, np.nan, 0.0, -0.0], np.float32)]
    return np.concatenate(pts).astype(np.float32)


@pytest.mark.parametrize("spec", TABLES)
def test_binary_search_locate_matches_index_map(spec):
    import paper_1510_02975_amd as P
    library()
    dev = device()
    func, p, a, b, N, part, vals = spec
    t = P.pwl_build(func, p, a, b, N, part, vals)
    xh = _points(t, a, b)
    x = torch.from_numpy(xh).to(dev)
    with locate_mode(P, P.LOCATE_MAP):
        y_map = P.pwl_eval(t, x).cpu().numpy()
        seg_map = P.pwl_locate(t, x).cpu().numpy()
    with locate_mode(P, P.LOCATE_SEARCH):
        y_bs = P.pwl_eval(t, x).cpu().numpy()
        seg_bs = P.pwl_locate(t, x).cpu().numpy()
        y_bs_odd = P.pwl_eval(t, x[1:4000]).cpu().numpy()   # scalar (misaligned) path
    say("  f=%d N=%d: %d points" % (func, N, x.numel()))
    d = P.pwl_table_download(t)
    Xg, vg = d["knots"].astype(np.float64), d["values"].astype(np.float64)
    fin = ~np.isnan(xh)
    ref_seg = O.locate(Xg, xh[fin].astype(np.float64))
    assert np.array_equal(seg_map[fin], ref_seg)
    assert np.array_equal(seg_bs[fin], ref_seg)
    assert np.all(seg_bs[~fin] == 0) and np.all(seg_map[~fin] == 0)
    y_ref = O.evaluate(Xg, vg, xh.astype(np.float64))
    scale = fmax_abs(func, p, a, b)
    assert np.array_equal(np.isnan(y_bs), np.isnan(y_ref))
    assert np.max(np.abs(y_bs[fin] - y_ref[fin])) <= Y_TOL * scale
    assert np.array_equal(y_map, y_bs, equal_nan=True)
    assert np.array_equal(y_map[1:4000], y_bs_odd, equal_nan=True)
    t.free()


@pytest.mark.parametrize("spec", TABLES)
def test_record_layouts_match_oracle(spec):
    """Structure-of-arrays records and value/slope pairs against the oracle
    and bit-identical to the packed records, with the index map and with the
    binary search; also on the scalar (misaligned) path and with a
    vertex-value override."""
    import paper_1510_02975_amd as P
    library()
    dev = device()
    func, p, a, b, N, part, vals = spec
    t = P.pwl_build(func, p, a, b, N, part, vals)
    xh = _points(t, a, b)
    x = torch.from_numpy(xh).to(dev)
    d = P.pwl_table_download(t)
    Xg, vg = d["knots"].astype(np.float64), d["values"].astype(np.float64)
    vo = torch.from_numpy((1.0 + 0.5 * np.cos(np.arange(N + 1))).astype(np.float32)).to(dev)
    out = {}
    for rec in (P.RECORDS_PACKED, P.RECORDS_SOA, P.RECORDS_PAIRS):
        for mode in (P.LOCATE_MAP, P.LOCATE_SEARCH):
            with records_layout(P, rec), locate_mode(P, mode):
                out[rec, mode] = (P.pwl_eval(t, x).cpu().numpy(), P.pwl_eval(t, x[1:4000]).cpu().numpy(),
                                  P.pwl_eval(t, x, v_override=vo).cpu().numpy())
    say("  f=%d N=%d: %d points, 6 variants" % (func, N, x.numel()))
    fin = ~np.isnan(xh)
    y_ref = O.evaluate(Xg, vg, xh.astype(np.float64))
    scale = fmax_abs(func, p, a, b)
    y_vo_ref = O.evaluate(Xg, vo.cpu().numpy().astype(np.float64), xh.astype(np.float64))
    for rec in (P.RECORDS_SOA, P.RECORDS_PAIRS):
        y_rec = out[rec, P.LOCATE_MAP][0]
        assert np.array_equal(np.isnan(y_rec), np.isnan(y_ref))
        assert np.max(np.abs(y_rec[fin] - y_ref[fin])) <= Y_TOL * scale
        y_vo = out[rec, P.LOCATE_MAP][2]
        assert np.max(np.abs(y_vo[fin] - y_vo_ref[fin])) <= 4e-6 * 1.5
    base = out[P.RECORDS_PACKED, P.LOCATE_MAP]
    for key, val in out.items():
        for a_, b_ in zip(base, val):
            assert np.array_equal(a_, b_, equal_nan=True), key
    t.free()
