"""Minimal ctypes access to HIP events (libamdhip64) for kernel timing."""
from __future__ import annotations

import ctypes as C
import os

_hip = None


def hip():
    global _hip
    if _hip is None:
        for name in ("libamdhip64.so", "/opt/rocm/lib/libamdhip64.so"):
            try:
                _hip = C.CDLL(name)
                break
            except OSError:
                continue
        if _hip is None:
            raise OSError("libamdhip64.so not found")
        _hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        _hip.hipEventDestroy.argtypes = [C.c_void_p]
        _hip.hipEventSynchronize.argtypes = [C.c_void_p]
        _hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        _hip.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
    return _hip


class EventPool:
    """A pool of (start, stop) HIP event pairs."""

    def __init__(self, n_pairs: int):
        self.pairs = []
        for _ in range(n_pairs):
            a, b = C.c_void_p(), C.c_void_p()
            if hip().hipEventCreate(C.byref(a)) or hip().hipEventCreate(C.byref(b)):
                raise RuntimeError("hipEventCreate failed")
            self.pairs.append((a.value, b.value))
        self.used = 0

    def next(self):
        if self.used == len(self.pairs):          # grow on demand
            a, b = C.c_void_p(), C.c_void_p()
            if hip().hipEventCreate(C.byref(a)) or hip().hipEventCreate(C.byref(b)):
                raise RuntimeError("hipEventCreate failed")
            self.pairs.append((a.value, b.value))
        p = self.pairs[self.used]
        self.used += 1
        return p

    def elapsed_ms(self):
        """Durations (ms) of every pair used so far."""
        out = []
        for a, b in self.pairs[: self.used]:
            hip().hipEventSynchronize(b)
            ms = C.c_float(0.0)
            if hip().hipEventElapsedTime(C.byref(ms), a, b):
                raise RuntimeError("hipEventElapsedTime failed")
            out.append(ms.value)
        return out

    def reset(self):
        self.used = 0

    def close(self):
        for a, b in self.pairs:
            hip().hipEventDestroy(a)
            hip().hipEventDestroy(b)
        self.pairs = []


def record(event: int, stream: int) -> None:
    if hip().hipEventRecord(event, stream):
        raise RuntimeError("hipEventRecord failed")
