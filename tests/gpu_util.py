"""Helpers shared by the tests: the built library, the device, and the
oracle-side tolerances (written here so every test states the same bar)."""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Parity tolerances of the path: outputs within 2e-6 max|f| of the FP64 oracle, table
# values within 1e-6 max|f|, gradients within 1e-5 relative.
Y_TOL = 2e-6
VALUE_TOL = 1e-6
GRAD_TOL = 1e-5


def library():
    """The HIP library, built in place if nothing is built yet."""
    import paper_1510_02975_amd as P
    from paper_1510_02975_amd import build as B
    if not os.path.exists(P.binding.LIB_PATH):
        B.build()
    return P.load_library()


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    return torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)


def fmax_abs(func, params, a, b):
    """max |f| on [a, b] from a dense sample (tolerance scale)."""
    import oracle as O
    t = np.linspace(a, b, 200001)
    return float(np.max(np.abs(O.f_value(func, params, t))))


def ulp_diff32(a, b):
    """Distance in FP32 ulps between two arrays of FP32 values."""
    ia = np.asarray(a, dtype=np.float32).view(np.int32).astype(np.int64)
    ib = np.asarray(b, dtype=np.float32).view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return np.abs(ia - ib)


class locate_mode:
    """Run a block with pwl_set_locate(mode), then restore the mode in force
    before (the library may run a tuned mode, not the default)."""

    def __init__(self, P, mode):
        self.P, self.mode = P, mode

    def __enter__(self):
        self.prev = self.P.pwl_get_locate()
        self.P.pwl_set_locate(self.mode)

    def __exit__(self, *exc):
        self.P.pwl_set_locate(self.prev)


class launch_shape:
    """Run a block with pwl_set_launch(kernel, *shape), then restore the
    shape in force before."""

    def __init__(self, P, kernel, shape):
        self.P, self.kernel, self.shape = P, kernel, shape

    def __enter__(self):
        self.prev = self.P.pwl_get_launch(self.kernel)
        self.P.pwl_set_launch(self.kernel, *self.shape)

    def __exit__(self, *exc):
        self.P.pwl_set_launch(self.kernel, *self.prev)


class records_layout:
    """Run a block with pwl_set_records(layout), then restore the layout in
    force before."""

    def __init__(self, P, layout):
        self.P, self.layout = P, layout

    def __enter__(self):
        self.prev = self.P.pwl_get_records()
        self.P.pwl_set_records(self.layout)

    def __exit__(self, *exc):
        self.P.pwl_set_records(self.prev)
