"""The paper's own GPU locate - a branch-free binary search over the knots
(Sec. IV-V), here over the knots staged in LDS - against the default index
map: both must give the same segment, so pwl_eval's outputs are
bit-identical, on random points, every knot and its FP32 neighbours, the
domain ends, points outside, +-inf and NaN."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import device, library, say

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


@pytest.mark.parametrize("spec", TABLES)
def test_binary_search_locate_matches_index_map(spec):
    import paper_1510_02975_amd as P
    library()
    dev = device()
    func, p, a, b, N, part, vals = spec
    t = P.pwl_build(func, p, a, b, N, part, vals)
    X = P.pwl_table_download(t)["knots"]
    pts = [W.uniform_points(a - 1.0, b + 1.0, 100003, 3),
           X, np.nextafter(X, np.float32(-np.inf)), np.nextafter(X, np.float32(np.inf)),
           np.array([a, b, -np.inf, np.inf, np.nan, 0.0, -0.0], np.float32)]
    x = torch.from_numpy(np.concatenate(pts).astype(np.float32)).to(dev)
    assert P.pwl_get_locate() == P.LOCATE_MAP
    y_map = P.pwl_eval(t, x).cpu().numpy()
    P.pwl_set_locate(P.LOCATE_SEARCH)
    try:
        y_bs = P.pwl_eval(t, x).cpu().numpy()
        y_bs_odd = P.pwl_eval(t, x[1:4000]).cpu().numpy()   # scalar (misaligned) path
    finally:
        P.pwl_set_locate(P.LOCATE_MAP)
    say("  f=%d N=%d: %d points" % (func, N, x.numel()))
    assert np.array_equal(y_map, y_bs, equal_nan=True)
    assert np.array_equal(y_map[1:4000], y_bs_odd, equal_nan=True)
    t.free()
