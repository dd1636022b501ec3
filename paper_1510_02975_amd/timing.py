"""Kernel timing shared by the benchmark and the autotuner: HIP events that
take no system-scope fence, and back-to-back launches after a time-based
warm-up.

A default HIP event writes back and invalidates the caches when it is
recorded; events created with hipEventDisableSystemFence do neither, so they
do not sit between the kernels they separate.  The GPU raises its clocks
under sustained load: a warm-up counted in launches times the ramp, so the
warm-up here is counted in seconds."""

import ctypes
import time

import numpy as np

WARM_SECONDS = 0.25   # sustained load before each timed phase
_DISABLE_SYSTEM_FENCE = 0x20000000


class Marks:
    """`count` timing-only HIP events on torch's current (or a given)
    stream.  The HIP runtime is the one torch loaded (same soname), so
    torch's stream handles are valid here."""

    def __init__(self, torch, count):
        self.torch = torch
        self.hip = ctypes.CDLL("libamdhip64.so.7")
        self.hip.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = []
        for _ in range(count):
            e = ctypes.c_void_p()
            self._check(self.hip.hipEventCreateWithFlags(ctypes.byref(e), _DISABLE_SYSTEM_FENCE))
            self.ev.append(e)

    @staticmethod
    def _check(rc):
        if rc != 0:
            raise RuntimeError("HIP event call failed with status %d" % rc)

    def record(self, i, stream=None):
        s = stream if stream is not None else self.torch.cuda.current_stream()
        self._check(self.hip.hipEventRecord(self.ev[i], s.cuda_stream))

    def ms(self, i, j):
        out = ctypes.c_float()
        self._check(self.hip.hipEventElapsedTime(ctypes.byref(out), self.ev[i], self.ev[j]))
        return out.value

    def free(self):
        for e in self.ev:
            self.hip.hipEventDestroy(e)
        self.ev = []


def warm_up(torch, fn, seconds=WARM_SECONDS, min_calls=0):
    """Run fn(i) until `seconds` of sustained load have passed (and at least
    min_calls calls); returns the seconds spent."""
    t0 = time.perf_counter()
    i = 0
    while i < min_calls or time.perf_counter() - t0 < seconds:
        fn(i)
        i += 1
        if i % 8 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def launch_durations(torch, fn, reps=20, warm_seconds=WARM_SECONDS):
    """Durations (s) of `reps` back-to-back launches fn(0..reps-1) on the
    current stream, each between two fence-free events, after warm_seconds
    of sustained load."""
    warm_up(torch, fn, warm_seconds)
    m = Marks(torch, reps + 1)
    for i in range(reps):
        m.record(i)
        fn(i)
    m.record(reps)
    torch.cuda.synchronize()
    d = np.array([m.ms(i, i + 1) for i in range(reps)]) * 1e-3
    m.free()
    return d


def timed_median(torch, fn, reps=20, warm_seconds=WARM_SECONDS):
    """Median duration (s) of back-to-back launches (see launch_durations)."""
    return float(np.median(launch_durations(torch, fn, reps, warm_seconds)))
