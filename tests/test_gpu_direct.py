"""The no-table baseline pwl_direct_eval (FP32 device math) against the FP64
oracle's f: within 1e-6 max|f| for every built-in function, on vector and
scalar (misaligned) paths."""

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from tests.gpu_util import device, fmax_abs, library

pytestmark = pytest.mark.gpu

FUNCS = [
    (O.GAUSSIAN, (1.3, 2.0), -6.0, 6.0),
    (O.LORENTZIAN, (0.7, 1.0), -20.0, 20.0),
    (O.BESSEL_J0, (1.0,), 0.0, 50.0),
    (O.POLY, (1.0, -0.5, 0.25, 0.0, 0.01, 0.0), -3.0, 3.0),
    (O.EXP, (0.5, 1.0), -4.0, 4.0),
]


@pytest.mark.parametrize("spec", FUNCS)
def test_direct_eval_matches_oracle(spec):
    import paper_1510_02975_amd as P
    library()
    dev = device()
    func, p, a, b = spec
    x_h = W.uniform_points(a, b, 100003, 6)
    x = torch.from_numpy(x_h).to(dev)
    y = P.pwl_direct_eval(func, p, x).cpu().numpy().astype(np.float64)
    y_odd = P.pwl_direct_eval(func, p, x[1:]).cpu().numpy().astype(np.float64)
    ref = O.f_value(func, p, x_h.astype(np.float64))
    fm = fmax_abs(func, p, a, b)
    assert np.max(np.abs(y - ref)) <= 1e-6 * fm
    assert np.array_equal(y[1:], y_odd)
