"""ctypes wrapper of the CPU oracle (oracle.c).  TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The GPU library never links or calls it; the two share
no code.  See oracle.c for what each function computes and which passage of
the thesis it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

CLASS_NAMES = ("003", "012", "102", "021D", "021U", "021C", "111D", "111U",
               "030T", "030C", "201", "120D", "120U", "120C", "210", "300")

_lib = None


def build() -> str:
    """Compile liboracle.so with gcc (always recompiles)."""
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O3", "-std=gnu11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
           SRC_PATH, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_table.argtypes = [ctypes.c_void_p]
    lib.oracle_table.restype = ctypes.c_int
    lib.oracle_graph_new.argtypes = [i32, i64, vp, vp]
    lib.oracle_graph_new.restype = vp
    lib.oracle_graph_free.argtypes = [vp]
    lib.oracle_graph_free.restype = None
    lib.oracle_graph_arcs.argtypes = [vp]
    lib.oracle_graph_arcs.restype = i64
    lib.oracle_graph_degree.argtypes = [vp, i32]
    lib.oracle_graph_degree.restype = i64
    lib.oracle_census.argtypes = [vp, u64p]
    lib.oracle_census.restype = ctypes.c_int
    lib.oracle_census_range.argtypes = [vp, i32, i32, u64p]
    lib.oracle_census_range.restype = ctypes.c_int
    lib.oracle_census_mt.argtypes = [vp, ctypes.c_int, u64p]
    lib.oracle_census_mt.restype = ctypes.c_int
    lib.oracle_census64.argtypes = [vp, u64p]
    lib.oracle_census64.restype = ctypes.c_int
    lib.oracle_brute.argtypes = [i32, i64, vp, vp, ctypes.c_int, u64p]
    lib.oracle_brute.restype = ctypes.c_int
    _lib = lib
    return lib


def _arcs(src, dst):
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    if s.shape != d.shape:
        raise ValueError("src and dst differ in length")
    return s, d


def table() -> np.ndarray:
    """The 64-entry TriadTable (class index 0..15 per 6-bit TriadCode)."""
    t = np.zeros(64, np.uint8)
    if _load().oracle_table(t.ctypes.data) != 0:
        raise RuntimeError("class definitions do not partition the 64 codes")
    return t


class OracleGraph:
    """The oracle's own canonicalised adjacency (sorted out-lists and
    neighbour lists) for repeated census calls."""

    def __init__(self, n: int, src, dst):
        lib = _load()
        self._s, self._d = _arcs(src, dst)
        self.n = int(n)
        h = lib.oracle_graph_new(self.n, self._s.size, self._s.ctypes.data, self._d.ctypes.data)
        if not h:
            raise ValueError("bad arc list (id out of range) or out of memory")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _load().oracle_graph_free(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def arcs(self) -> int:
        return int(_load().oracle_graph_arcs(self._h))

    def degree(self, u: int) -> int:
        return int(_load().oracle_graph_degree(self._h, u))

    def census(self) -> np.ndarray:
        out = np.zeros(16, np.uint64)
        if _load().oracle_census(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))) != 0:
            raise MemoryError
        return out

    def census_range(self, u0: int, u1: int) -> np.ndarray:
        out = np.zeros(16, np.uint64)
        if _load().oracle_census_range(self._h, u0, u1,
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))) != 0:
            raise MemoryError
        return out

    def census64(self) -> np.ndarray:
        out = np.zeros(64, np.uint64)
        if _load().oracle_census64(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))) != 0:
            raise MemoryError
        return out

    def census_mt(self, threads: int) -> np.ndarray:
        out = np.zeros(16, np.uint64)
        r = _load().oracle_census_mt(self._h, threads, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        if r < 0:
            raise MemoryError
        return out


def census(n: int, src, dst) -> np.ndarray:
    """Full 16-class census of the digraph (n, src->dst)."""
    with OracleGraph(n, src, dst) as g:
        return g.census()


def census64(n: int, src, dst) -> np.ndarray:
    """64-class labelled census: raw TriadCode histogram in the loop's roles."""
    with OracleGraph(n, src, dst) as g:
        return g.census64()


def brute(n: int, src, dst, threads: int = 1) -> np.ndarray:
    """Naive O(n^3) census over every triple."""
    s, d = _arcs(src, dst)
    out = np.zeros(16, np.uint64)
    r = _load().oracle_brute(int(n), s.size, s.ctypes.data, d.ctypes.data, int(threads),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if r != 0:
        raise ValueError("bad arc list or out of memory")
    return out
