"""CPU checks of the C ABI: the library loads, exports every entry point that
include/pwl.h declares, and rejects invalid arguments on the host before any
device work (no compute call is made here)."""

import ctypes
import os
import re

import pytest

from tests.gpu_util import ROOT, library


def header_symbols():
    text = open(os.path.join(ROOT, "include", "pwl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pwl_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = header_symbols()
    for s in ["pwl_build", "pwl_eval", "pwl_eval_backward", "pwl_table_download", "pwl_table_free",
              "pwl_last_error", "pwl_locate", "pwl_rebuild", "pwl_table_check", "pwl_table_info"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    lib = library()
    missing = [s for s in header_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_abi_version():
    assert library().pwl_abi_version() == 2


def _build(lib, func=0, params=None, n=0, a=-1.0, b=1.0, N=8, part=1, vals=1):
    out = ctypes.c_void_p(123)
    arr = (ctypes.c_double * max(1, len(params or [])))(*(params or [])) if params else None
    st = lib.pwl_build(func, arr, n, a, b, N, part, vals, None, ctypes.byref(out))
    return st, out


@pytest.mark.parametrize("kw,status", [
    (dict(N=0), -1),
    (dict(N=-3), -1),
    (dict(N=4097), -5),
    (dict(a=1.0, b=1.0), -1),
    (dict(a=2.0, b=1.0), -1),
    (dict(a=float("nan")), -1),
    (dict(b=float("inf")), -1),
    (dict(a=1.0, b=1.0 + 1e-9), -1),          # equal after rounding to FP32
    (dict(func=5), -1),
    (dict(part=2), -1),
    (dict(vals=7), -1),
    (dict(params=[1.0, 2.0, 3.0], n=3), -1),  # Gaussian takes at most 2
    (dict(params=[-1.0], n=1), -1),           # width must be > 0
    (dict(params=[float("nan")], n=1), -1),
    (dict(func=2, params=[1.0, 2.0], n=2), -1),
    (dict(n=7), -1),
])
def test_build_rejects_invalid_arguments_on_host(kw, status):
    lib = library()
    st, out = _build(lib, **kw)
    assert st == status
    assert out.value is None            # *out cleared, nothing allocated
    assert len(lib.pwl_last_error()) > 0


def test_build_null_out():
    lib = library()
    assert lib.pwl_build(0, None, 0, -1.0, 1.0, 8, 1, 1, None, None) == -1


def test_calls_on_null_table_are_rejected():
    lib = library()
    assert lib.pwl_eval(None, None, None, None, 10, None) == -1
    assert lib.pwl_eval_backward(None, None, None, None, None, None, None, 10, None) == -1
    assert lib.pwl_locate(None, None, None, 10, None) == -1
    assert lib.pwl_table_info(None, None, None, None, None, None, None, None) == -1
    assert lib.pwl_table_check(None, None, None) == -1
    assert lib.pwl_table_download(None, None, None, None, None, None) == -1
    assert lib.pwl_rebuild(None, 0, None, 0, -1.0, 1.0, 1, 1, None) == -1
    lib.pwl_table_free(None)   # no-op


def test_baseline_argument_checks():
    lib = library()
    assert lib.pwl_direct_gaussian(None, None, -1, 1.0, 1.0, 0, None) == -1
    assert lib.pwl_direct_gaussian(None, None, 4, 0.0, 1.0, 0, None) == -1
    assert lib.pwl_direct_gaussian(None, None, 4, 1.0, 1.0, 0, None) == -1
    assert lib.pwl_direct_gaussian(None, None, 0, 1.0, 1.0, 0, None) == 0   # n = 0 does nothing
    assert lib.pwl_copy(None, None, -2, None) == -1
    assert lib.pwl_copy(None, None, 0, None) == 0
    assert lib.pwl_copy(None, None, 5, None) == -1


def test_python_binding_names_match_the_abi():
    import paper_1510_02975_amd as P
    for s in header_symbols():
        assert hasattr(P, s), s


def test_binding_rejects_host_tensors():
    import torch
    import paper_1510_02975_amd as P
    with pytest.raises((ValueError, TypeError)):
        P.binding._ptr(torch.zeros(4), name="x")
    with pytest.raises(TypeError):
        P.binding._ptr(torch.zeros(4, dtype=torch.float64), name="x")


def test_batch_create_rejects_invalid_arguments_on_host():
    lib = library()
    out = ctypes.c_void_p(5)
    offs = (ctypes.c_int64 * 3)(0, 4, 2)
    tabs = (ctypes.c_void_p * 2)(1, 2)
    assert lib.pwl_batch_create(tabs, 2, offs, None, ctypes.byref(out)) == -1   # decreasing offsets
    assert out.value is None
    offs = (ctypes.c_int64 * 3)(1, 4, 8)
    assert lib.pwl_batch_create(tabs, 2, offs, None, ctypes.byref(out)) == -1   # offsets[0] != 0
    offs = (ctypes.c_int64 * 3)(0, 4, 8)
    assert lib.pwl_batch_create(tabs, 0, offs, None, ctypes.byref(out)) == -1   # T < 1
    nulls = (ctypes.c_void_p * 2)(None, None)
    assert lib.pwl_batch_create(nulls, 2, offs, None, ctypes.byref(out)) == -1  # NULL table
    assert lib.pwl_batch_create(tabs, 2, offs, None, None) == -1
    assert lib.pwl_batch_eval(None, None, None, None) == -1
    assert lib.pwl_batch_eval_backward(None, None, None, None, None, None, None) == -1
    assert lib.pwl_batch_replay(None, None) == -1
    assert lib.pwl_batch_info(None, None, None, None, None, None, None, None) == -1
    lib.pwl_batch_free(None)


def test_set_launch_validation():
    lib = library()
    assert lib.pwl_set_launch(0, 3, 256, 2) == -1
    assert lib.pwl_set_launch(0, 2, 100, 2) == -1
    assert lib.pwl_set_launch(0, 2, 256, 0) == -1
    assert lib.pwl_set_launch(7, 2, 256, 2) == -1
    u, b, w = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    assert lib.pwl_get_launch(0, ctypes.byref(u), ctypes.byref(b), ctypes.byref(w)) == 0
    assert lib.pwl_set_launch(0, 1, 128, 3) == 0
    u2 = ctypes.c_int32()
    lib.pwl_get_launch(0, ctypes.byref(u2), None, None)
    assert u2.value == 1
    assert lib.pwl_set_launch(0, 0, 0, 0) == 0            # defaults back
    lib.pwl_get_launch(0, ctypes.byref(u2), None, None)
    assert u2.value == u.value


def test_plan_tol_rejects_invalid_arguments_on_host():
    lib = library()
    n, part, pred = ctypes.c_int32(-7), ctypes.c_int32(-7), ctypes.c_double(-1.0)
    p = (ctypes.c_double * 2)(1.0, 1.0)
    args = lambda tol, norm, vals, a=-5.0, b=5.0, func=0: lib.pwl_plan_tol(
        func, p, 2, a, b, tol, norm, vals, None, ctypes.byref(n), ctypes.byref(part), ctypes.byref(pred))
    assert args(0.0, 0, 1) == -1                  # tol must be > 0
    assert args(-1e-3, 0, 1) == -1
    assert args(float("nan"), 0, 1) == -1
    assert args(float("inf"), 0, 1) == -1
    assert args(1e-3, 2, 1) == -1                 # unknown norm
    assert args(1e-3, 0, 5) == -1                 # unknown values kind
    assert args(1e-3, 0, 1, a=1.0, b=1.0) == -1   # empty domain
    assert args(1e-3, 0, 1, func=99) == -1        # unknown function
    assert n.value == -7 and part.value == -7 and pred.value == -1.0
    out = ctypes.c_void_p(5)
    assert lib.pwl_build_tol(0, p, 2, -5.0, 5.0, 0.0, 0, 1, None, ctypes.byref(out)) == -1
    assert out.value is None
    assert lib.pwl_build_tol(0, p, 2, -5.0, 5.0, 1e-3, 0, 1, None, None) == -1


def test_set_locate_validation():
    lib = library()
    assert lib.pwl_set_locate(7) == -1
    assert lib.pwl_set_locate(-1) == -1
    assert lib.pwl_get_locate() == 0
    assert lib.pwl_set_locate(1) == 0 and lib.pwl_get_locate() == 1
    assert lib.pwl_set_locate(0) == 0 and lib.pwl_get_locate() == 0


def test_build_sampled_rejects_invalid_arguments_on_host():
    lib = library()
    out = ctypes.c_void_p(5)
    f = ctypes.c_void_p(16)    # never dereferenced: validation fails first
    assert lib.pwl_build_sampled(None, f, 8, 0.0, 1.0, 16, 1, 1, None, ctypes.byref(out)) == -1
    assert lib.pwl_build_sampled(f, None, 8, 0.0, 1.0, 16, 1, 1, None, ctypes.byref(out)) == -1
    assert lib.pwl_build_sampled(f, f, 0, 0.0, 1.0, 16, 1, 1, None, ctypes.byref(out)) == -1
    assert lib.pwl_build_sampled(f, f, 8, 1.0, 1.0, 16, 1, 1, None, ctypes.byref(out)) == -1
    assert lib.pwl_build_sampled(f, f, 8, 0.0, 1.0, 0, 1, 1, None, ctypes.byref(out)) == -1
    assert lib.pwl_build_sampled(f, f, 8, 0.0, 1.0, 16, 9, 1, None, ctypes.byref(out)) == -1
    assert out.value is None
    assert lib.pwl_build_sampled(f, f, 8, 0.0, 1.0, 16, 1, 1, None, None) == -1
    # the sampled id is not a parameterised function
    p = (ctypes.c_double * 1)(1.0)
    assert lib.pwl_build(32, p, 1, 0.0, 1.0, 16, 1, 1, None, ctypes.byref(out)) == -1


def test_kde_rejects_invalid_arguments_on_host():
    lib = library()
    buf = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    s = (ctypes.c_float * 3)(6.0, 6.0, 6.0)
    bad_s = (ctypes.c_float * 3)(6.0, 0.0, 6.0)
    assert lib.pwl_kde(None, 3, buf, buf, 8, 8, 2, 1, s, buf, None) == -1      # mode
    assert lib.pwl_kde(None, 1, buf, buf, 0, 8, 2, 1, s, buf, None) == -1      # H
    assert lib.pwl_kde(None, 1, buf, buf, 8, 8, 0, 1, s, buf, None) == -1      # T
    assert lib.pwl_kde(None, 1, buf, buf, 8, 8, 2, 33, s, buf, None) == -1     # radius
    assert lib.pwl_kde(None, 1, buf, buf, 8, 8, 2, 1, bad_s, buf, None) == -1  # sigma
    assert lib.pwl_kde(None, 1, None, buf, 8, 8, 2, 1, s, buf, None) == -1     # frame
    assert lib.pwl_kde(None, 0, buf, buf, 8, 8, 2, 1, s, buf, None) == -1      # table mode, no table
