"""ctypes binding of libtc_cpu.so (include/tc_cpu.h): the multicore CPU census
kept as a context baseline.  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtc_cpu.so")
_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1603_02655_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        lib.tc_cpu_census.restype = ctypes.c_int
        lib.tc_cpu_census.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        _lib = lib
    return _lib


def census(n: int, src, dst, threads: int = 0) -> tuple[np.ndarray, float]:
    """(16 counts, census seconds) of the digraph (n, src -> dst)."""
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    if s.shape != d.shape:
        raise ValueError("src and dst differ in length")
    out = np.zeros(16, np.uint64)
    secs = ctypes.c_double(0.0)
    rc = load().tc_cpu_census(int(n), s.size, s.ctypes.data, d.ctypes.data, int(threads), out.ctypes.data,
                              ctypes.byref(secs))
    if rc != 0:
        raise ValueError("tc_cpu_census: bad arguments (null pointer, negative size or id out of range)")
    return out, secs.value
