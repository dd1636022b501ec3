"""Tables built from a target error (pwl_plan_tol / pwl_build_tol): the N
and partition the GPU chooses agree with the FP64 oracle's predictions
(Results 4-6, Sec. III-B2, and the L-infinity estimates), N - 1 would miss
the target, and the table the GPU then builds meets it, checked by oracle
quadrature on the downloaded table (the predictions are asymptotic: within
5% once N >= 256, 15% below; 10% / 20% for the L-infinity error of the
projection).  The tolerances stay well above the FP32 floor of the tables:
their vertex values carry ~1e-7 max|f| (the projection's FP32 hat
quadrature up to ~2e-7), which at tol = 1e-6 max|f| alone adds up to 20%."""

import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import device, library, say

pytestmark = pytest.mark.gpu

CASES = [
    # func, params, a, b, tol, norm, values
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 1e-5, 0, O.INTERP),
    (O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 3e-6, 1, O.PROJ),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 1e-5, 1, O.PROJ),
    (O.LORENTZIAN, (1.0, 1.0), -20.0, 20.0, 2e-5, 0, O.INTERP),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 1e-5, 0, O.PROJ),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0, 1e-4, 1, O.INTERP),
    (O.POLY, (0.0, 0.0, 0.5), -1.0, 1.0, 1e-4, 1, O.INTERP),   # x^2 / 2: f'' constant
]


def _oracle_needs(func, p, a, b, tol, norm, vals):
    """{partition: smallest N whose predicted error is <= tol}."""
    key = "l2" if norm == 0 else "linf"
    out = {}
    for part in (O.UNIFORM, O.OPTIMAL):
        c = O.predicted_errors(func, p, a, b, 1)[key][(part, vals)]   # error = c / N^2
        out[part] = max(1, math.ceil(math.sqrt(c / tol)))
    return out


@pytest.mark.parametrize("case", CASES)
def test_plan_matches_oracle_and_table_meets_tol(case):
    import paper_1510_02975_amd as P
    library()
    device()
    func, p, a, b, tol, norm, vals = case
    N, part, pred = P.pwl_plan_tol(func, p, a, b, tol, norm, vals)
    need = _oracle_needs(func, p, a, b, tol, norm, vals)
    n_or = min(need.values())
    say("  f=%d tol=%g norm=%s vals=%d: GPU N=%d partition %d (predicted %.3e); oracle N uniform %d, optimal %d"
        % (func, tol, "L2" if norm == 0 else "Linf", vals, N, part, pred, need[O.UNIFORM], need[O.OPTIMAL]))
    assert abs(N - n_or) <= 1            # the integrals differ in the last digits only
    if abs(need[O.UNIFORM] - need[O.OPTIMAL]) > 1:
        # a clear winner: the GPU picks it (the optimal partition only when it needs fewer segments)
        assert part == min(need, key=lambda k: (need[k], k))
    assert pred <= tol * (1 + 1e-9)
    key = "l2" if norm == 0 else "linf"
    c_gpu = O.predicted_errors(func, p, a, b, 1)[key][(part, vals)]
    if N > 1:
        assert c_gpu / (N - 1) ** 2 > tol * (1 - 1e-6)   # N - 1 would miss the target
    t = P.pwl_build_tol(func, p, a, b, tol, norm, vals)
    d = P.pwl_table_download(t)
    X, v = d["knots"].astype(np.float64), d["values64"]
    err = O.l2_error(func, p, X, v) if norm == 0 else O.linf_error(func, p, X, v)
    # L-infinity of the projection: the estimate takes each element's own
    # minimiser, while the projection couples neighbouring elements; its
    # maximum error runs up to ~7% above the estimate here (N ~ 750)
    loose = norm == 1 and vals == O.PROJ
    slack = (1.10 if loose else 1.05) if N >= 256 else (1.20 if loose else 1.15)
    say("    built N=%d: error %.3e (%.3f of tol)" % (t.N, err, err / tol))
    assert t.N == N
    assert err <= slack * tol
    t.free()


def test_affine_function_needs_one_segment():
    import paper_1510_02975_amd as P
    library()
    device()
    N, part, pred = P.pwl_plan_tol(O.POLY, (1.0, 2.0), -3.0, 4.0, 1e-9, 0, O.PROJ)
    assert N == 1 and pred == 0.0


def test_unreachable_tolerance_reports_capacity():
    import paper_1510_02975_amd as P
    library()
    device()
    with pytest.raises(P.PWLError) as e:
        P.pwl_plan_tol(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 1e-14, 0, O.PROJ)
    assert e.value.status == -5
