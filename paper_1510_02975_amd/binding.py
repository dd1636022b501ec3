"""Thin ctypes binding over libpwl.so (the C ABI in include/pwl.h).

Each pwl_* function here has the name and argument order of the C entry
point; it only marshals arguments (tensor data pointers, the current HIP
stream) and turns a negative status into an exception.  All arithmetic runs
in the HIP kernels.  PyTorch supplies device memory and streams.
"""

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpwl.so")
# Launch shapes and locate mode chosen by the autotuner on MI355X
# (autotune.py writes it), applied when the library is loaded; the
# environment variable PWL_TUNED=0 keeps the library's built-in defaults.
TUNED_PATH = os.path.join(_PKG, "tuned_mi355x.json")
TUNED_SOURCE = None   # description of the applied tuning, or None

GAUSSIAN, LORENTZIAN, BESSEL_J0, POLY, EXP, SAMPLED = 0, 1, 2, 16, 17, 32
UNIFORM, OPTIMAL = 0, 1
INTERP, PROJ = 0, 1
FLAG_DEGENERATE, FLAG_KNOTS_COLLAPSED, FLAG_NONFINITE = 1, 2, 4
NORM_L2, NORM_LINF = 0, 1
MAX_N = 4096

STATUS = {0: "PWL_OK", -1: "PWL_EINVAL", -2: "PWL_ENOMEM", -3: "PWL_EHIP", -4: "PWL_EKNOTS",
          -5: "PWL_ECAPACITY"}


class PWLError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS.get(status, status), message))
        self.status = status


_lib = None

_c_int32 = ctypes.c_int32
_c_int64 = ctypes.c_int64
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int32)

_SIGNATURES = {
    "pwl_build": (_c_int32, [_c_int32, _dp, _c_int32, ctypes.c_double, ctypes.c_double, _c_int32,
                             _c_int32, _c_int32, _vp, ctypes.POINTER(_vp)]),
    "pwl_rebuild": (_c_int32, [_vp, _c_int32, _dp, _c_int32, ctypes.c_double, ctypes.c_double,
                               _c_int32, _c_int32, _vp]),
    "pwl_build_sampled": (_c_int32, [_vp, _vp, _c_int32, ctypes.c_double, ctypes.c_double, _c_int32, _c_int32,
                                     _c_int32, _vp, ctypes.POINTER(_vp)]),
    "pwl_plan_tol": (_c_int32, [_c_int32, _dp, _c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                _c_int32, _c_int32, _vp, _ip, _ip, _dp]),
    "pwl_build_tol": (_c_int32, [_c_int32, _dp, _c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 _c_int32, _c_int32, _vp, ctypes.POINTER(_vp)]),
    "pwl_table_check": (_c_int32, [_vp, _vp, _ip]),
    "pwl_table_info": (_c_int32, [_vp, _ip, _dp, _dp, _ip, _ip, _ip, _ip]),
    "pwl_table_download": (_c_int32, [_vp, _fp, _fp, _dp, _dp, _vp]),
    "pwl_table_free": (None, [_vp]),
    "pwl_eval": (_c_int32, [_vp, _vp, _vp, _vp, _c_int64, _vp]),
    "pwl_eval_backward": (_c_int32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _c_int64, _vp]),
    "pwl_eval_backward_noalloc": (_c_int32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _c_int64, _vp]),
    "pwl_locate": (_c_int32, [_vp, _vp, _vp, _c_int64, _vp]),
    "pwl_direct_gaussian": (_c_int32, [_vp, _vp, _c_int64, ctypes.c_float, ctypes.c_float, _c_int32, _vp]),
    "pwl_copy": (_c_int32, [_vp, _vp, _c_int64, _vp]),
    "pwl_direct_eval": (_c_int32, [_c_int32, _dp, _c_int32, _vp, _vp, _c_int64, _vp]),
    "pwl_kde": (_c_int32, [_vp, _c_int32, _vp, _vp, _c_int32, _c_int32, _c_int32, _c_int32, _fp, _vp, _vp]),
    "pwl_batch_create": (_c_int32, [ctypes.POINTER(_vp), _c_int32, ctypes.POINTER(_c_int64), _vp,
                                    ctypes.POINTER(_vp)]),
    "pwl_batch_eval": (_c_int32, [_vp, _vp, _vp, _vp]),
    "pwl_batch_eval_backward": (_c_int32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pwl_batch_capture": (_c_int32, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pwl_batch_replay": (_c_int32, [_vp, _vp]),
    "pwl_batch_info": (_c_int32, [_vp, _ip, ctypes.POINTER(_c_int64), ctypes.POINTER(_c_int64), _ip, _ip, _ip, _ip]),
    "pwl_batch_free": (None, [_vp]),
    "pwl_set_launch": (_c_int32, [_c_int32, _c_int32, _c_int32, _c_int32]),
    "pwl_get_launch": (_c_int32, [_c_int32, _ip, _ip, _ip]),
    "pwl_set_locate": (_c_int32, [_c_int32]),
    "pwl_get_locate": (_c_int32, []),
    "pwl_set_records": (_c_int32, [_c_int32]),
    "pwl_get_records": (_c_int32, []),
    "pwl_last_error": (ctypes.c_char_p, []),
    "pwl_abi_version": (_c_int32, []),
}


def load_library(path=None):
    """Load libpwl.so (once).  Raises if the HIP library has not been built:
    there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError("libpwl.so is not built (expected at %s); run "
                          "`python -m paper_1510_02975_amd.build`" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    if os.environ.get("PWL_TUNED", "1") != "0":
        apply_tuned(TUNED_PATH)
    return lib


def apply_tuned(path):
    """Install the launch shapes and locate mode of an autotuner result file
    (see autotune.save); a missing file leaves the library defaults."""
    global TUNED_SOURCE
    import json
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    for k, shape in rec.get("launch", {}).items():
        _check(_lib.pwl_set_launch(int(k), *[int(v) for v in shape]))
    if "locate" in rec:
        _check(_lib.pwl_set_locate(int(rec["locate"])))
    if "records" in rec:
        _check(_lib.pwl_set_records(int(rec["records"])))
    TUNED_SOURCE = rec.get("source", os.path.basename(path))
    return rec


def _check(status):
    if status != 0:
        msg = load_library().pwl_last_error()
        raise PWLError(status, msg.decode() if msg else "")


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t, dtype=torch.float32, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _params(params):
    params = [] if params is None else [float(p) for p in params]
    arr = (ctypes.c_double * max(len(params), 1))(*params) if params else None
    return arr, len(params)


class Table:
    """Owner of a pwl_table handle."""

    def __init__(self, handle, func, params, a, b, N, partition, values):
        self.handle = handle
        self.func, self.params = func, tuple(params) if params else ()
        self.N, self.partition, self.values = N, partition, values
        self.a, self.b = self.info()[1:3]

    @property
    def _as_parameter_(self):
        return self.handle

    def info(self):
        lib = load_library()
        N, part, vals, K = _c_int32(), _c_int32(), _c_int32(), _c_int32()
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib.pwl_table_info(self.handle, ctypes.byref(N), ctypes.byref(a), ctypes.byref(b),
                                  ctypes.byref(part), ctypes.byref(vals), ctypes.byref(K), None))
        return N.value, a.value, b.value, part.value, vals.value, K.value

    def flags(self):
        """Build flags (PWL_FLAG_*) of the table's last build; waits for it."""
        f = _c_int32()
        _check(load_library().pwl_table_info(self.handle, None, None, None, None, None, None, ctypes.byref(f)))
        return f.value

    def free(self):
        if self.handle is not None:
            load_library().pwl_table_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Entry points, same names as the C ABI.
# ---------------------------------------------------------------------------

def pwl_build(func, params, a, b, N, partition=OPTIMAL, values=PROJ, stream=None, check=True):
    """Build a table on the current device; returns a Table.  With check the
    stream is synchronised and a knot collapse raises PWLError."""
    lib = load_library()
    arr, npar = _params(params)
    out = ctypes.c_void_p()
    _check(lib.pwl_build(int(func), arr, npar, float(a), float(b), int(N), int(partition), int(values),
                         _stream(stream), ctypes.byref(out)))
    t = Table(out, func, params, a, b, int(N), partition, values)
    if check:
        pwl_table_check(t, stream)
    return t


def pwl_build_sampled(f, f2, a, b, N, partition=OPTIMAL, values=PROJ, stream=None, check=True):
    """Table for the function sampled as f[i], f2[i] = f(t_i), f''(t_i) at
    t_i = a + i (b - a) / S (device FP64 tensors of S + 1 values).  With
    check the stream is synchronised, so the samples may be freed after."""
    if f.dtype != torch.float64 or f2.dtype != torch.float64:
        raise TypeError("samples must be float64")
    if f.numel() != f2.numel() or f.numel() < 2:
        raise ValueError("f and f2 need the same number (>= 2) of samples")
    lib = load_library()
    out = ctypes.c_void_p()
    _check(lib.pwl_build_sampled(_ptr(f, torch.float64, "f"), _ptr(f2, torch.float64, "f2"), f.numel() - 1,
                                 float(a), float(b), int(N), int(partition), int(values), _stream(stream),
                                 ctypes.byref(out)))
    t = Table(out, SAMPLED, None, a, b, int(N), partition, values)
    if check:
        pwl_table_check(t, stream)
    return t


def pwl_plan_tol(func, params, a, b, tol, norm=NORM_L2, values=PROJ, stream=None):
    """(N, partition, predicted error) that reach `tol` in `norm`."""
    lib = load_library()
    arr, npar = _params(params)
    N, part, pred = _c_int32(), _c_int32(), ctypes.c_double()
    _check(lib.pwl_plan_tol(int(func), arr, npar, float(a), float(b), float(tol), int(norm), int(values),
                            _stream(stream), ctypes.byref(N), ctypes.byref(part), ctypes.byref(pred)))
    return N.value, part.value, pred.value


def pwl_build_tol(func, params, a, b, tol, norm=NORM_L2, values=PROJ, stream=None, check=True):
    """Build the table pwl_plan_tol chooses; returns a Table."""
    N, part, _ = pwl_plan_tol(func, params, a, b, tol, norm, values, stream)
    lib = load_library()
    arr, npar = _params(params)
    out = ctypes.c_void_p()
    _check(lib.pwl_build_tol(int(func), arr, npar, float(a), float(b), float(tol), int(norm), int(values),
                             _stream(stream), ctypes.byref(out)))
    t = Table(out, func, params, a, b, N, part, values)
    if check:
        pwl_table_check(t, stream)
    return t


def pwl_rebuild(table, func, params, a, b, partition=OPTIMAL, values=PROJ, stream=None):
    lib = load_library()
    arr, npar = _params(params)
    _check(lib.pwl_rebuild(table.handle, int(func), arr, npar, float(a), float(b), int(partition),
                           int(values), _stream(stream)))
    table.func, table.params, table.partition, table.values = func, tuple(params or ()), partition, values


def pwl_table_check(table, stream=None):
    """Synchronise and return the build flags; raises PWLError on knot collapse."""
    flags = _c_int32()
    _check(load_library().pwl_table_check(table.handle, _stream(stream), ctypes.byref(flags)))
    return flags.value


def pwl_table_info(table):
    return table.info()


def pwl_table_download(table, stream=None):
    """Host copies: dict of numpy arrays knots (f32), values (f32), knots64, values64."""
    import numpy as np
    n1 = table.N + 1
    k32 = np.empty(n1, np.float32)
    v32 = np.empty(n1, np.float32)
    k64 = np.empty(n1, np.float64)
    v64 = np.empty(n1, np.float64)
    _check(load_library().pwl_table_download(
        table.handle, k32.ctypes.data_as(_fp), v32.ctypes.data_as(_fp), k64.ctypes.data_as(_dp),
        v64.ctypes.data_as(_dp), _stream(stream)))
    return {"knots": k32, "values": v32, "knots64": k64, "values64": v64}


def pwl_table_free(table):
    table.free()


def pwl_eval(table, x, y=None, v_override=None, stream=None):
    if y is None:
        y = torch.empty_like(x)
    if y.numel() != x.numel():
        raise ValueError("y must have as many elements as x")
    if v_override is not None and v_override.numel() != table.N + 1:
        raise ValueError("v_override must have N + 1 elements")
    _check(load_library().pwl_eval(table.handle, _ptr(v_override, name="v_override"), _ptr(x, name="x"),
                                   _ptr(y, name="y"), x.numel(), _stream(stream)))
    return y


def pwl_eval_backward(table, x, g, y=None, dx=None, dv=None, v_override=None, stream=None,
                      want=("y", "dx", "dv")):
    """Fused forward + backward; returns (y, dx, dv) with None for outputs not wanted."""
    if g.numel() != x.numel():
        raise ValueError("g must have as many elements as x")
    if y is None and "y" in want:
        y = torch.empty_like(x)
    if dx is None and "dx" in want:
        dx = torch.empty_like(x)
    if dv is None and "dv" in want:
        dv = torch.empty(table.N + 1, dtype=torch.float32, device=x.device)
    if v_override is not None and v_override.numel() != table.N + 1:
        raise ValueError("v_override must have N + 1 elements")
    if dv is not None and dv.numel() != table.N + 1:
        raise ValueError("dv must have N + 1 elements")
    _check(load_library().pwl_eval_backward(
        table.handle, _ptr(v_override, name="v_override"), _ptr(x, name="x"), _ptr(g, name="g"),
        _ptr(y, name="y"), _ptr(dx, name="dx"), _ptr(dv, name="dv"), x.numel(), _stream(stream)))
    return y, dx, dv


def pwl_eval_backward_noalloc(table, x, g, y, dx, dv, v_override=None, stream=None):
    """pwl_eval_backward with the dL/dv partial sums in the library's fixed
    device scratch: the caller passes every output it wants (None for the
    others) and nothing is allocated."""
    if g.numel() != x.numel():
        raise ValueError("g must have as many elements as x")
    for name, a in (("y", y), ("dx", dx)):
        if a is not None and a.numel() != x.numel():
            raise ValueError("%s must have as many elements as x" % name)
    if v_override is not None and v_override.numel() != table.N + 1:
        raise ValueError("v_override must have N + 1 elements")
    if dv is not None and dv.numel() != table.N + 1:
        raise ValueError("dv must have N + 1 elements")
    _check(load_library().pwl_eval_backward_noalloc(
        table.handle, _ptr(v_override, name="v_override"), _ptr(x, name="x"), _ptr(g, name="g"),
        _ptr(y, name="y"), _ptr(dx, name="dx"), _ptr(dv, name="dv"), x.numel(), _stream(stream)))
    return y, dx, dv


def pwl_locate(table, x, seg=None, stream=None):
    if seg is None:
        seg = torch.empty(x.shape, dtype=torch.int32, device=x.device)
    _check(load_library().pwl_locate(table.handle, _ptr(x, name="x"), _ptr(seg, torch.int32, "seg"),
                                     x.numel(), _stream(stream)))
    return seg


def pwl_direct_gaussian(x, y=None, s=1.0, amp=1.0, fast=False, stream=None):
    if y is None:
        y = torch.empty_like(x)
    _check(load_library().pwl_direct_gaussian(_ptr(x, name="x"), _ptr(y, name="y"), x.numel(), float(s),
                                              float(amp), int(bool(fast)), _stream(stream)))
    return y


def pwl_copy(src, dst=None, stream=None):
    if dst is None:
        dst = torch.empty_like(src)
    _check(load_library().pwl_copy(_ptr(src, name="src"), _ptr(dst, name="dst"), src.numel(),
                                   _stream(stream)))
    return dst


class Batch:
    """Owner of a pwl_batch handle; keeps its tables alive."""

    def __init__(self, handle, tables, offsets):
        self.handle = handle
        self.tables = list(tables)
        self.offsets = list(int(o) for o in offsets)
        self.T, self.npoints, self.dv_len, self.grid_fwd, self.grid_bwd, self.runs_fwd, self.runs_bwd = \
            self.info()
        self.dv_offsets = [0]
        for t in self.tables:
            self.dv_offsets.append(self.dv_offsets[-1] + t.N + 1)

    def info(self):
        T, gf, gb, rf, rb = _c_int32(), _c_int32(), _c_int32(), _c_int32(), _c_int32()
        n, d = _c_int64(), _c_int64()
        _check(load_library().pwl_batch_info(self.handle, ctypes.byref(T), ctypes.byref(n), ctypes.byref(d),
                                             ctypes.byref(gf), ctypes.byref(gb), ctypes.byref(rf),
                                             ctypes.byref(rb)))
        return T.value, n.value, d.value, gf.value, gb.value, rf.value, rb.value

    def free(self):
        if self.handle is not None:
            load_library().pwl_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def pwl_batch_create(tables, offsets, stream=None):
    """tables: list of Table; offsets: T+1 point offsets (host)."""
    T = len(tables)
    if len(offsets) != T + 1:
        raise ValueError("offsets must have T + 1 entries")
    handles = (_vp * T)(*[t.handle for t in tables])
    offs = (_c_int64 * (T + 1))(*[int(o) for o in offsets])
    out = _vp()
    _check(load_library().pwl_batch_create(handles, T, offs, _stream(stream), ctypes.byref(out)))
    return Batch(out, tables, offsets)


def pwl_batch_eval(batch, x, y=None, stream=None):
    if x.numel() != batch.npoints:
        raise ValueError("x must hold the batch's %d points" % batch.npoints)
    if y is None:
        y = torch.empty_like(x)
    _check(load_library().pwl_batch_eval(batch.handle, _ptr(x, name="x"), _ptr(y, name="y"), _stream(stream)))
    return y


def pwl_batch_eval_backward(batch, x, g, y=None, dx=None, dv=None, stream=None, want=("y", "dx")):
    if x.numel() != batch.npoints or g.numel() != batch.npoints:
        raise ValueError("x and g must hold the batch's %d points" % batch.npoints)
    if y is None and "y" in want:
        y = torch.empty_like(x)
    if dx is None and "dx" in want:
        dx = torch.empty_like(x)
    if dv is None:
        dv = torch.empty(batch.dv_len, dtype=torch.float32, device=x.device)
    _check(load_library().pwl_batch_eval_backward(
        batch.handle, _ptr(x, name="x"), _ptr(g, name="g"), _ptr(y, name="y"), _ptr(dx, name="dx"),
        _ptr(dv, name="dv"), _stream(stream)))
    return y, dx, dv


def pwl_batch_capture(batch, x, y=None, g=None, dx=None, dv=None, stream=None):
    _check(load_library().pwl_batch_capture(
        batch.handle, _ptr(x, name="x"), _ptr(g, name="g"), _ptr(y, name="y"), _ptr(dx, name="dx"),
        _ptr(dv, name="dv"), _stream(stream)))


def pwl_batch_replay(batch, stream=None):
    _check(load_library().pwl_batch_replay(batch.handle, _stream(stream)))


def pwl_batch_info(batch):
    return batch.info()


def pwl_batch_free(batch):
    batch.free()


KERNEL_FORWARD, KERNEL_BACKWARD, KERNEL_BATCH, KERNEL_BATCH_BACKWARD = 0, 1, 2, 3


def pwl_set_launch(kernel, unroll=0, block=0, wg_per_cu=0):
    """Set the launch shape of a kernel family (all zeros: defaults)."""
    _check(load_library().pwl_set_launch(int(kernel), int(unroll), int(block), int(wg_per_cu)))


def pwl_get_launch(kernel):
    u, b, w = _c_int32(), _c_int32(), _c_int32()
    _check(load_library().pwl_get_launch(int(kernel), ctypes.byref(u), ctypes.byref(b), ctypes.byref(w)))
    return u.value, b.value, w.value


LOCATE_MAP, LOCATE_SEARCH = 0, 1
RECORDS_PACKED, RECORDS_SOA, RECORDS_PAIRS = 0, 1, 2
KDE_TABLE, KDE_EXPF, KDE_FAST_EXPF = 0, 1, 2


def pwl_direct_eval(func, params, x, y=None, stream=None):
    """y = f(x) in FP32 with the device math library (no table)."""
    if y is None:
        y = torch.empty_like(x)
    if y.numel() != x.numel():
        raise ValueError("y must have as many elements as x")
    arr, npar = _params(params)
    _check(load_library().pwl_direct_eval(int(func), arr, npar, _ptr(x, name="x"), _ptr(y, name="y"), x.numel(),
                                          _stream(stream)))
    return y


def pwl_kde(table, mode, frame, hist, radius, sigma, out=None, stream=None):
    """Per-pixel sums of Gaussian kernels: frame uint8 [H, W, 4], hist uint8
    [T, H, W, 4] (device); returns FP32 [H, W]."""
    if frame.dtype != torch.uint8 or hist.dtype != torch.uint8:
        raise TypeError("frame and hist must be uint8 RGBA")
    if frame.dim() != 3 or frame.shape[2] != 4 or hist.dim() != 4 or tuple(hist.shape[1:]) != tuple(frame.shape):
        raise ValueError("need frame [H, W, 4] and hist [T, H, W, 4]")
    H, W = int(frame.shape[0]), int(frame.shape[1])
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=frame.device)
    sig = (ctypes.c_float * 3)(*[float(s) for s in sigma])
    _check(load_library().pwl_kde(table.handle if table is not None else None, int(mode),
                                  _ptr(frame, torch.uint8, "frame"), _ptr(hist, torch.uint8, "hist"), H, W,
                                  int(hist.shape[0]), int(radius), sig, _ptr(out, name="out"), _stream(stream)))
    return out


def pwl_set_locate(mode):
    _check(load_library().pwl_set_locate(int(mode)))


def pwl_get_locate():
    return int(load_library().pwl_get_locate())


def pwl_set_records(layout):
    _check(load_library().pwl_set_records(int(layout)))


def pwl_get_records():
    return int(load_library().pwl_get_records())


def pwl_last_error():
    m = load_library().pwl_last_error()
    return m.decode() if m else ""


def pwl_abi_version():
    return load_library().pwl_abi_version()


# ---------------------------------------------------------------------------
# Autograd
# ---------------------------------------------------------------------------

class PWLFunction(torch.autograd.Function):
    """y = v(x) for the CPWL table with vertex values `values` (a [N+1] FP32
    tensor, typically a Parameter); backward gives dL/dx and dL/dvalues from
    the fused HIP kernel."""

    @staticmethod
    def forward(ctx, x, values, table):
        x = x.contiguous()
        values = values.contiguous()
        ctx.table = table
        ctx.save_for_backward(x, values)
        return pwl_eval(table, x, v_override=values)

    @staticmethod
    def backward(ctx, gy):
        x, values = ctx.saved_tensors
        table = ctx.table
        gy = gy.contiguous()
        need_x, need_v = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        want = tuple(w for w, need in (("dx", need_x), ("dv", need_v)) if need)
        if not want:
            return None, None, None
        _, dx, dv = pwl_eval_backward(table, x, gy, v_override=values, want=want)
        return dx, dv, None


class PWLTable(torch.nn.Module):
    """A CPWL approximation of f with trainable vertex values."""

    def __init__(self, func, params, a, b, N, partition=OPTIMAL, values=PROJ, device=None):
        super().__init__()
        if device is not None:
            torch.cuda.set_device(device)
        self.table = pwl_build(func, params, a, b, N, partition, values)
        v = torch.from_numpy(pwl_table_download(self.table)["values"]).cuda()
        self.values = torch.nn.Parameter(v)

    def forward(self, x):
        return PWLFunction.apply(x, self.values, self.table)
