"""GPU table construction against the FP64 oracle (through the C ABI).

Knots: the GPU's FP64 scan sums in a different order than the oracle's
sequential one, so FP32 knots may differ by at most one ulp (in practice they
are identical).  Values: FP32 f and FP32 Gauss-Legendre sums on the GPU, FP64
solve; compared with the oracle evaluated on the GPU's own FP32 knots to
1e-6 max|f|.
"""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import VALUE_TOL, device, fmax_abs, library, locate_mode, say, ulp_diff32

pytestmark = pytest.mark.gpu

CASES = [
    # func, params, a, b, N, partition
    (O.GAUSSIAN, (1.0, 1.0), -4.0, 4.0, 64, O.UNIFORM),
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 1024, O.OPTIMAL),
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 512, O.OPTIMAL),
    (O.GAUSSIAN, (0.1, 2.0), -0.5, 0.5, 16, O.UNIFORM),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 256, O.OPTIMAL),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 4096, O.OPTIMAL),
    (O.LORENTZIAN, (3.7, 1.0), -74.0, 74.0, 16, O.UNIFORM),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 1024, O.OPTIMAL),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 4096, O.OPTIMAL),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 17, O.UNIFORM),
    (O.EXP, (1.3, 0.5), -1.0, 2.0, 100, O.OPTIMAL),
    (O.POLY, (0.5, -1.0, 3.0), -2.0, 7.0, 90, O.OPTIMAL),
    (O.GAUSSIAN, (1.0, 1.0), -3.0, 2.0, 1, O.OPTIMAL),
    (O.GAUSSIAN, (1.0, 1.0), -3.0, 2.0, 2, O.OPTIMAL),
    (O.GAUSSIAN, (1.0, 1.0), -3.0, 2.0, 3, O.UNIFORM),
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 7, O.OPTIMAL),
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 2048, O.OPTIMAL),
]


def _ids(c):
    return "f%d-N%d-p%d" % (c[0], c[4], c[5])


def _gpu_table(P, func, params, a, b, N, part, vals):
    device()
    t = P.pwl_build(func, params, a, b, N, part, vals)
    d = P.pwl_table_download(t)
    flags = P.pwl_table_check(t)
    return t, d, flags


@pytest.mark.parametrize("case", CASES, ids=[_ids(c) for c in CASES])
@pytest.mark.parametrize("vals", [O.INTERP, O.PROJ])
def test_table_matches_oracle(case, vals):
    import paper_1510_02975_amd as P
    library()
    func, params, a, b, N, part = case
    say("build parity %s vals=%d" % (_ids(case), vals))
    t, d, flags = _gpu_table(P, func, params, a, b, N, part, vals)
    ref = O.build_table(func, params, a, b, N, part, vals)
    assert flags == ref["flags"]
    # knots: at most one FP32 ulp apart (differently ordered FP64 scans)
    ku = ulp_diff32(d["knots"], ref["X"])
    assert ku.max() <= 1, (ku.max(), np.argmax(ku))
    assert d["knots"][0] == np.float32(ref["a"]) and d["knots"][-1] == np.float32(ref["b"])
    assert np.all(np.diff(d["knots"].astype(np.float64)) > 0)
    if part == O.OPTIMAL:
        assert np.max(np.abs(d["knots64"] - ref["X64"])) <= 1e-9 * (b - a)
    # values against the oracle on the GPU's own knots
    X = d["knots"].astype(np.float64)
    vref = O.interp_values(func, params, X) if vals == O.INTERP else O.proj_values(func, params, X)
    scale = fmax_abs(func, params, a, b)
    err32 = np.max(np.abs(d["values"].astype(np.float64) - vref))
    err64 = np.max(np.abs(d["values64"] - vref))
    say("  max|dv| fp32 %.3e fp64 %.3e (scale %.3e)" % (err32, err64, scale))
    assert err32 <= VALUE_TOL * scale
    assert err64 <= VALUE_TOL * scale
    if vals == O.INTERP:
        assert np.array_equal(d["values64"], d["values"].astype(np.float64))
    t.free()


def test_knot_collapse_reports_and_evaluates_to_nan():
    import paper_1510_02975_amd as P
    import torch
    library()
    device()
    a = 1.0
    b = float(np.nextafter(np.nextafter(np.float32(1.0), np.float32(2)), np.float32(2)))
    t = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), a, b, 64, O.OPTIMAL, O.PROJ, check=False)
    assert t.flags() & P.FLAG_KNOTS_COLLAPSED          # pwl_table_info waits for the build
    with pytest.raises(P.PWLError) as ei:
        P.pwl_table_check(t)
    assert ei.value.status == -4
    x = torch.tensor([1.0, 1.0000001, 0.5, 3.0], device="cuda")
    y = P.pwl_eval(t, x)
    assert torch.isnan(y).all()
    t.free()


def test_degenerate_function_falls_back_to_uniform():
    import paper_1510_02975_amd as P
    library()
    t, d, flags = _gpu_table(P, O.POLY, (1.0, -2.0), -1.0, 3.0, 40, O.OPTIMAL, O.PROJ)
    assert flags == P.FLAG_DEGENERATE
    assert t.flags() == P.FLAG_DEGENERATE            # the same word through pwl_table_info
    U, _ = O.uniform_knots(-1.0, 3.0, 40)
    assert np.array_equal(d["knots"].astype(np.float64), U)
    assert np.max(np.abs(d["values64"] - (1.0 - 2.0 * U))) <= 1e-6
    t.free()


def test_rebuild_in_place_matches_fresh_build():
    import paper_1510_02975_amd as P
    library()
    device()
    t = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 256, O.UNIFORM, O.INTERP)
    P.pwl_rebuild(t, O.LORENTZIAN, (2.0, 1.5), -30.0, 30.0, O.OPTIMAL, O.PROJ)
    assert t.flags() == 0
    assert P.pwl_table_check(t) == 0
    d1 = P.pwl_table_download(t)
    t2 = P.pwl_build(O.LORENTZIAN, (2.0, 1.5), -30.0, 30.0, 256, O.OPTIMAL, O.PROJ)
    d2 = P.pwl_table_download(t2)
    for k in ("knots", "values", "knots64", "values64"):
        assert np.array_equal(d1[k], d2[k]), k
    assert t.info() == t2.info()
    t.free()
    t2.free()


def test_build_capacity_and_domain_rounding():
    import paper_1510_02975_amd as P
    library()
    device()
    with pytest.raises(P.PWLError) as ei:
        P.pwl_build(O.GAUSSIAN, None, -1.0, 1.0, 5000)
    assert ei.value.status == -5
    t = P.pwl_build(O.GAUSSIAN, None, -0.1, 0.3, 8, O.UNIFORM, O.INTERP)
    N, a, b, part, vals, K = t.info()
    assert a == float(np.float32(-0.1)) and b == float(np.float32(0.3)) and N == 8
    t.free()


@pytest.mark.parametrize("case", [
    # func, params, a, b, N, partition, expected map cells / N
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 1024, O.OPTIMAL, 8),   # knots crowd at 0: 2.2 per 4N-cell
    (O.LORENTZIAN, (0.1, 1.0), -2.0, 2.0, 256, O.OPTIMAL, 8),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 4096, O.OPTIMAL, 4),   # 8N would not fit in LDS
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 1024, O.OPTIMAL, 4),       # 0.56 per 4N-cell
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 1024, O.OPTIMAL, 4),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 1024, O.UNIFORM, 2),
])
def test_map_size_per_table(case):
    """The index map gets 8N cells where the optimal knots crowd (more than
    1.5 predicted per 4N-cell at the density's peak, N <= 2048), 4N otherwise
    and 2N for a uniform partition; whatever its size, the forward equals
    the binary-search locate bit for bit on every knot and its neighbours."""
    import paper_1510_02975_amd as P
    library()
    dev = device()
    func, p, a, b, N, part, ratio = case
    t = P.pwl_build(func, p, a, b, N, part, O.PROJ)
    assert t.info()[5] == ratio * N
    X = P.pwl_table_download(t)["knots"]
    x = torch.from_numpy(np.concatenate([X, np.nextafter(X, np.float32(-np.inf)), np.nextafter(X, np.float32(np.inf)),
                                         W.uniform_points(a, b, 50001, 9)]).astype(np.float32)).to(dev)
    with locate_mode(P, P.LOCATE_MAP):
        y = P.pwl_eval(t, x)
    with locate_mode(P, P.LOCATE_SEARCH):
        y_bs = P.pwl_eval(t, x)
    assert torch.equal(y, y_bs)
    t.free()
