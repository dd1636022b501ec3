"""Tables built from samples of f and f'' (pwl_build_sampled) against the FP64
oracle built from the same samples (the cubic spline with those values and
second derivatives): FP32 knots within 1 ulp, vertex values within
1e-6 max|f|, evaluation within 2e-6 max|f|; the samples may be freed once
the build has run; a table from samples of the Gaussian evaluates like the
table of the Gaussian itself."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import VALUE_TOL, Y_TOL, device, library, say, ulp_diff32

pytestmark = pytest.mark.gpu


def _gauss(t):
    return np.exp(-t * t / 2.0), (t * t - 1.0) * np.exp(-t * t / 2.0)


def _wave(t):
    """sin(3t) exp(-t^2/4) + t/10 and its second derivative (calculus)."""
    s, c, e = np.sin(3 * t), np.cos(3 * t), np.exp(-t * t / 4)
    return s * e + 0.1 * t, e * (-9 * s - 3 * t * c + (t * t / 4 - 0.5) * s)


CASES = [
    ("gauss", _gauss, -5.0, 5.0, 4096, 512, O.OPTIMAL, O.PROJ),
    ("gauss", _gauss, -5.0, 5.0, 97, 64, O.UNIFORM, O.INTERP),
    ("wave", _wave, -6.0, 6.0, 2000, 1000, O.OPTIMAL, O.PROJ),
    ("wave", _wave, -6.0, 6.0, 300, 300, O.OPTIMAL, O.INTERP),
    ("wave", _wave, -6.0, 6.0, 1, 16, O.UNIFORM, O.PROJ),
]


@pytest.mark.parametrize("case", CASES, ids=["%s-S%d-N%d-p%d-v%d" % (c[0], c[4], c[5], c[6], c[7]) for c in CASES])
def test_sampled_table_matches_oracle(case):
    import paper_1510_02975_amd as P
    library()
    dev = device()
    name, fn, a, b, S, N, part, vals = case
    t_s = a + (b - a) * np.arange(S + 1) / S
    f_h, f2_h = fn(t_s)
    f_d = torch.from_numpy(f_h).to(dev)
    f2_d = torch.from_numpy(f2_h).to(dev)
    t = P.pwl_build_sampled(f_d, f2_d, a, b, N, part, vals)     # synchronises
    del f_d, f2_d                                                # the table no longer needs them
    torch.cuda.synchronize()
    d = P.pwl_table_download(t)
    smp = O.Samples(f_h, f2_h, a, b)
    ref = O.build_table(O.SAMPLED, smp, a, b, N, part, vals)
    fmax = float(np.max(np.abs(O.f_value(O.SAMPLED, smp, np.linspace(a, b, 100001)))))
    assert int(ulp_diff32(d["knots"], ref["X"].astype(np.float32)).max()) <= 1
    X = d["knots"].astype(np.float64)
    v_own = O.proj_values(O.SAMPLED, smp, X) if vals == O.PROJ else O.interp_values(O.SAMPLED, smp, X)
    assert np.max(np.abs(d["values64"] - v_own)) <= VALUE_TOL * fmax
    x_h = W.uniform_points(a - 0.5, b + 0.5, 200003, 5)
    y = P.pwl_eval(t, torch.from_numpy(x_h).to(dev)).cpu().numpy().astype(np.float64)
    err = np.max(np.abs(y - O.evaluate(ref["X"], ref["v"], x_h.astype(np.float64)))) / fmax
    say("  %s S=%d N=%d: max |y - oracle| = %.2e max|f|" % (name, S, N, err))
    assert err <= Y_TOL
    t.free()


def test_samples_of_the_gaussian_give_the_gaussian_table():
    import paper_1510_02975_amd as P
    library()
    dev = device()
    S = 1 << 14
    f_h, f2_h = _gauss(-5.0 + 10.0 * np.arange(S + 1) / S)
    ts = P.pwl_build_sampled(torch.from_numpy(f_h).to(dev), torch.from_numpy(f2_h).to(dev), -5.0, 5.0, 1024,
                             O.OPTIMAL, O.PROJ)
    tf = P.pwl_build(O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, 1024, O.OPTIMAL, O.PROJ)
    x = torch.from_numpy(W.gauss_big_points(1 << 20)).to(dev)
    d = float((P.pwl_eval(ts, x) - P.pwl_eval(tf, x)).abs().max())
    say("  sampled vs analytic Gaussian tables: max |dy| = %.2e" % d)
    assert d <= 2 * Y_TOL
    # a table from samples cannot be rebuilt as an analytic one
    with pytest.raises(P.PWLError) as ei:
        P.pwl_rebuild(ts, O.GAUSSIAN, (1.0, 1.0), -5.0, 5.0, O.OPTIMAL, O.PROJ)
    assert ei.value.status == -1
    assert float((P.pwl_eval(ts, x) - P.pwl_eval(tf, x)).abs().max()) == d   # unchanged
    ts.free()
    tf.free()
