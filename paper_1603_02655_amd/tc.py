"""Thin ctypes binding of libtc (include/tc.h).

Argument marshalling only: every step of the census runs in the HIP library.
The functions keep the C names (tc_context_create, tc_build_graph, tc_census,
...); ``Context`` and ``Graph`` wrap the handles for convenience.  Host arrays
are numpy; device arrays are ``DeviceArray`` buffers (their pointers are passed
with TC_BUILD_DEVICE_PTRS).

Device buffers are allocated through the HIP runtime that libtc itself links
(ROCm's libamdhip64.so.7).  PyTorch-ROCm ships a second, bundled HIP runtime;
a process that initialises both finds no GPU from the second one, so torch
tensors are not handed to this library in-process.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtc.so")

TC_OK = 0
TC_ERR_ARG = -1
TC_ERR_RANGE = -2
TC_ERR_NOMEM = -3
TC_ERR_DEVICE = -4
TC_ERR_BUSY = -5
TC_ERR_NOT_FOUND = -6
TC_ERR_SHUTDOWN = -7

TC_NOALLOC_MAX_GRAPHS = 256

TC_BUILD_DEFAULT = 0
TC_BUILD_STRICT = 1
TC_BUILD_DEVICE_PTRS = 2

CLASS_NAMES = ("003", "012", "102", "021D", "021U", "021C", "111D", "111U",
               "030T", "030C", "201", "120D", "120U", "120C", "210", "300")
BUCKETS = ("lane", "wave", "group", "hub")
NB = len(BUCKETS)


class TcError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = load().tc_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class tc_graph_info(ctypes.Structure):
    _fields_ = [("arcs_in", ctypes.c_int64), ("arcs_kept", ctypes.c_int64),
                ("self_loops_dropped", ctypes.c_int64), ("duplicates_dropped", ctypes.c_int64),
                ("asym_dyads", ctypes.c_int64), ("mutual_dyads", ctypes.c_int64),
                ("max_degree", ctypes.c_int64), ("device_bytes", ctypes.c_uint64),
                ("sum_d2", ctypes.c_uint64), ("bucket_dyads", ctypes.c_uint64 * 4),
                ("bucket_cost", ctypes.c_uint64 * 4), ("hub_tasks", ctypes.c_uint64),
                ("hub_stream", ctypes.c_uint64), ("hub_staged", ctypes.c_uint64),
                ("fwd_entries", ctypes.c_uint64), ("tri_bucket_edges", ctypes.c_uint64 * 4),
                ("tri_bucket_cost", ctypes.c_uint64 * 4), ("tri_tasks", ctypes.c_uint64),
                ("tri_stream", ctypes.c_uint64), ("tri_staged", ctypes.c_uint64),
                ("hub_groups", ctypes.c_uint64), ("tri_groups", ctypes.c_uint64),
                ("hub_chunk", ctypes.c_uint64), ("tri_chunk", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        for k in ("bucket_dyads", "bucket_cost", "tri_bucket_edges", "tri_bucket_cost"):
            d[k] = list(getattr(self, k))
        return d


class tc_tuning(ctypes.Structure):
    _fields_ = [("t0", ctypes.c_uint32), ("t1", ctypes.c_uint32), ("lane_blocks", ctypes.c_uint32),
                ("wave_blocks", ctypes.c_uint32), ("group_blocks", ctypes.c_uint32),
                ("batch_blocks", ctypes.c_uint32), ("t_hub", ctypes.c_uint32), ("hub_blocks", ctypes.c_uint32),
                ("tri", ctypes.c_uint32), ("hub_tile", ctypes.c_uint32), ("wave_tile", ctypes.c_uint32),
                ("group_tile", ctypes.c_uint32), ("group_size", ctypes.c_uint32), ("batch_tile", ctypes.c_uint32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class tc_kernel_stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * 4), ("launches", ctypes.c_uint64 * 4),
                ("census_calls", ctypes.c_uint64), ("batch_ms", ctypes.c_double),
                ("batch_launches", ctypes.c_uint64), ("totals_ms", ctypes.c_double),
                ("totals_launches", ctypes.c_uint64)]


class tc_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("resident_graphs", ctypes.c_uint64), ("bytes_in_flight", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_admission_ms", ctypes.c_double),
                ("failed_rounds", ctypes.c_uint64), ("abandoned_rounds", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

# C signatures: name -> (restype, argtypes)
_vp, _i32, _i64, _u32, _u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_P = ctypes.POINTER
SIGNATURES = {
    "tc_context_create": (ctypes.c_int, [ctypes.c_int, _u64, _vp, _P(_vp)]),
    "tc_context_destroy": (ctypes.c_int, [_vp]),
    "tc_build_graph": (ctypes.c_int, [_vp, _i32, _i64, _vp, _vp, _u32, _P(_vp), _P(tc_graph_info)]),
    "tc_graph_get_info": (ctypes.c_int, [_vp, _vp, _P(tc_graph_info)]),
    "tc_graph_release": (ctypes.c_int, [_vp, _vp]),
    "tc_census": (ctypes.c_int, [_vp, _vp, _vp]),
    "tc_census_range": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp]),
    "tc_census_shard": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp]),
    "tc_census64": (ctypes.c_int, [_vp, _vp, _vp]),
    "tc_census_batch": (ctypes.c_int, [_vp, _vp, _i32, _vp]),
    "tc_census_each": (ctypes.c_int, [_vp, _vp, _i32, _vp]),
    "tc_census_each_noalloc": (ctypes.c_int, [_vp, _vp, _i32, _vp]),
    "tc_submit": (ctypes.c_int, [_vp, _vp, _P(_u64)]),
    "tc_submit_arcs": (ctypes.c_int, [_vp, _i32, _i64, _vp, _vp, _u32, _P(_u64)]),
    "tc_poll": (ctypes.c_int, [_vp, _u64, _vp, _P(ctypes.c_int)]),
    "tc_serve_stop": (ctypes.c_int, [_vp]),
    "tc_serve_set_watchdog_ms": (ctypes.c_int, [_vp, ctypes.c_double]),
    "tc_serve_get_stats": (ctypes.c_int, [_vp, _P(tc_serve_stats)]),
    "tc_serve_reset_stats": (ctypes.c_int, [_vp]),
    "tc_set_tuning": (ctypes.c_int, [_vp, _P(tc_tuning)]),
    "tc_get_tuning": (ctypes.c_int, [_vp, _P(tc_tuning)]),
    "tc_graph_rebucket": (ctypes.c_int, [_vp, _vp]),
    "tc_autotune": (ctypes.c_int, [_vp, _vp, _i32, ctypes.c_char_p, _P(tc_tuning)]),
    "tc_set_timing": (ctypes.c_int, [_vp, ctypes.c_int]),
    "tc_get_kernel_stats": (ctypes.c_int, [_vp, _P(tc_kernel_stats)]),
    "tc_reset_kernel_stats": (ctypes.c_int, [_vp]),
    "tc_class_table": (ctypes.c_int, [_vp]),
    "tc_status_string": (ctypes.c_char_p, [ctypes.c_int]),
}


def load() -> ctypes.CDLL:
    """Loads the in-tree libtc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1603_02655_amd/build.py "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != TC_OK:
        raise TcError(rc, what)


def tc_class_table() -> np.ndarray:
    t = np.zeros(64, np.uint8)
    _check(load().tc_class_table(t.ctypes.data), "tc_class_table")
    return t


def _u64_out(k: int) -> np.ndarray:
    return np.zeros(k, np.uint64)


_hip = None


def hip_runtime() -> ctypes.CDLL:
    """The HIP runtime libtc is linked against (already loaded with it)."""
    global _hip
    if _hip is None:
        load()
        h = ctypes.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        h.hipFree.argtypes = [ctypes.c_void_p]
        h.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        h.hipSetDevice.argtypes = [ctypes.c_int]
        _hip = h
    return _hip


def device_synchronize(device: int = 0):
    h = hip_runtime()
    if h.hipSetDevice(device) != 0 or h.hipDeviceSynchronize() != 0:
        raise RuntimeError("hipDeviceSynchronize failed")


class DeviceArray:
    """A device copy of a host numpy array (plumbing for TC_BUILD_DEVICE_PTRS)."""

    ptr = None

    def __init__(self, host, dtype=np.int32, device: int = 0):
        a = np.ascontiguousarray(host, dtype=dtype)
        h = hip_runtime()
        if h.hipSetDevice(device) != 0:
            raise RuntimeError("hipSetDevice failed")
        p = ctypes.c_void_p()
        if h.hipMalloc(ctypes.byref(p), max(1, a.nbytes)) != 0:
            raise MemoryError("hipMalloc failed")
        self.ptr, self.size, self.dtype, self.device = p.value, int(a.size), a.dtype, device
        if a.nbytes and h.hipMemcpy(p, a.ctypes.data, a.nbytes, 1) != 0:  # host to device
            self.free()
            raise RuntimeError("hipMemcpy failed")

    def free(self):
        if self.ptr:
            hip_runtime().hipFree(self.ptr)
            self.ptr = None

    __del__ = free


class Graph:
    """A resident device graph (tc_graph handle)."""

    def __init__(self, ctx: "Context", handle: int, n: int, info: tc_graph_info):
        self.ctx, self.handle, self.n, self.info = ctx, handle, n, info.as_dict()

    def release(self):
        if self.handle:
            _check(load().tc_graph_release(self.ctx.handle, self.handle), "tc_graph_release")
            self.handle = None

    def census(self) -> np.ndarray:
        return self.ctx.census(self)


class Context:
    """A tc_context on one HIP device, on its own stream or a given hipStream_t."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, stream=None):
        lib = load()
        h = ctypes.c_void_p()
        s = None
        if stream is not None:
            s = ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
        _check(lib.tc_context_create(device, hbm_budget_bytes, s, ctypes.byref(h)), "tc_context_create")
        self.handle = h.value
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            load().tc_context_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- graphs ----------------------------------------------------------
    def build_graph(self, n: int, src, dst, strict: bool = False) -> Graph:
        flags = TC_BUILD_STRICT if strict else TC_BUILD_DEFAULT
        if isinstance(src, DeviceArray) or isinstance(dst, DeviceArray):
            if not (isinstance(src, DeviceArray) and isinstance(dst, DeviceArray)):
                raise TypeError("src and dst must both be host arrays or both DeviceArray")
            if src.size != dst.size or src.dtype != np.int32 or dst.dtype != np.int32:
                raise TypeError("device arcs must be int32 arrays of equal length")
            flags |= TC_BUILD_DEVICE_PTRS
            m = src.size
            ptr_s, ptr_d = src.ptr, dst.ptr
            keep = (src, dst)
        else:
            src = np.ascontiguousarray(src, dtype=np.int32)
            dst = np.ascontiguousarray(dst, dtype=np.int32)
            if src.shape != dst.shape:
                raise ValueError("src and dst differ in length")
            m = int(src.size)
            ptr_s, ptr_d = src.ctypes.data, dst.ctypes.data
            keep = (src, dst)
        h = ctypes.c_void_p()
        info = tc_graph_info()
        rc = load().tc_build_graph(self.handle, int(n), m, ptr_s, ptr_d, flags, ctypes.byref(h), ctypes.byref(info))
        del keep
        _check(rc, "tc_build_graph")
        return Graph(self, h.value, int(n), info)

    # -- census ----------------------------------------------------------
    def census(self, g: Graph) -> np.ndarray:
        out = _u64_out(16)
        _check(load().tc_census(self.handle, g.handle, out.ctypes.data), "tc_census")
        return out

    def census64(self, g: Graph) -> np.ndarray:
        out = _u64_out(64)
        _check(load().tc_census64(self.handle, g.handle, out.ctypes.data), "tc_census64")
        return out

    def census_range(self, g: Graph, u0: int, u1: int) -> np.ndarray:
        out = _u64_out(16)
        _check(load().tc_census_range(self.handle, g.handle, int(u0), int(u1), out.ctypes.data), "tc_census_range")
        return out

    def census_shard(self, g: Graph, shard: int, nshards: int) -> np.ndarray:
        out = _u64_out(16)
        _check(load().tc_census_shard(self.handle, g.handle, int(shard), int(nshards), out.ctypes.data),
               "tc_census_shard")
        return out

    def _many(self, fn, graphs):
        hs = (ctypes.c_void_p * len(graphs))(*[g.handle for g in graphs])
        out = _u64_out(16 * len(graphs))
        _check(getattr(load(), fn)(self.handle, hs, len(graphs), out.ctypes.data), fn)
        return out.reshape(len(graphs), 16)

    def census_batch(self, graphs) -> np.ndarray:
        return self._many("tc_census_batch", list(graphs))

    def census_each(self, graphs) -> np.ndarray:
        return self._many("tc_census_each", list(graphs))

    def census_each_noalloc(self, graphs) -> np.ndarray:
        return self._many("tc_census_each_noalloc", list(graphs))

    # -- serving ---------------------------------------------------------
    def submit(self, g: Graph) -> int:
        t = ctypes.c_uint64()
        _check(load().tc_submit(self.handle, g.handle, ctypes.byref(t)), "tc_submit")
        return t.value

    def submit_arcs(self, n: int, src, dst, strict: bool = False) -> int:
        s = np.ascontiguousarray(src, dtype=np.int32)
        d = np.ascontiguousarray(dst, dtype=np.int32)
        if s.shape != d.shape:
            raise ValueError("src and dst differ in length")
        t = ctypes.c_uint64()
        _check(load().tc_submit_arcs(self.handle, int(n), int(s.size), s.ctypes.data, d.ctypes.data,
                                     TC_BUILD_STRICT if strict else 0, ctypes.byref(t)), "tc_submit_arcs")
        return t.value

    def poll(self, ticket: int):
        """Returns the 16 counts when the ticket is done, else None; raises
        TcError if the ticket finished with an error."""
        out = _u64_out(16)
        done = ctypes.c_int()
        rc = load().tc_poll(self.handle, ticket, out.ctypes.data, ctypes.byref(done))
        if rc != TC_OK and not (rc == TC_ERR_SHUTDOWN and not done.value):
            raise TcError(rc, "tc_poll")
        return out if done.value else None

    def serve_stop(self):
        _check(load().tc_serve_stop(self.handle), "tc_serve_stop")

    def serve_set_watchdog_ms(self, ms: float):
        _check(load().tc_serve_set_watchdog_ms(self.handle, float(ms)), "tc_serve_set_watchdog_ms")

    def serve_stats(self) -> dict:
        s = tc_serve_stats()
        _check(load().tc_serve_get_stats(self.handle, ctypes.byref(s)), "tc_serve_get_stats")
        return s.as_dict()

    def serve_reset_stats(self):
        _check(load().tc_serve_reset_stats(self.handle), "tc_serve_reset_stats")

    # -- tuning and timing -----------------------------------------------
    def get_tuning(self) -> dict:
        t = tc_tuning()
        _check(load().tc_get_tuning(self.handle, ctypes.byref(t)), "tc_get_tuning")
        return t.as_dict()

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = tc_tuning(**cur)
        _check(load().tc_set_tuning(self.handle, ctypes.byref(t)), "tc_set_tuning")

    def rebucket(self, g: Graph):
        _check(load().tc_graph_rebucket(self.handle, g.handle), "tc_graph_rebucket")
        info = tc_graph_info()
        _check(load().tc_graph_get_info(self.handle, g.handle, ctypes.byref(info)), "tc_graph_get_info")
        g.info = info.as_dict()

    def autotune(self, sample, cache_path: str | None = None) -> dict:
        hs = (ctypes.c_void_p * len(sample))(*[g.handle for g in sample])
        t = tc_tuning()
        cp = cache_path.encode() if cache_path else None
        _check(load().tc_autotune(self.handle, hs, len(sample), cp, ctypes.byref(t)), "tc_autotune")
        return t.as_dict()

    def set_timing(self, enable: bool = True):
        _check(load().tc_set_timing(self.handle, 1 if enable else 0), "tc_set_timing")

    def kernel_stats(self) -> dict:
        s = tc_kernel_stats()
        _check(load().tc_get_kernel_stats(self.handle, ctypes.byref(s)), "tc_get_kernel_stats")
        return {"ms": list(s.ms), "launches": list(s.launches), "census_calls": s.census_calls,
                "batch_ms": s.batch_ms, "batch_launches": s.batch_launches,
                "totals_ms": s.totals_ms, "totals_launches": s.totals_launches}

    def reset_kernel_stats(self):
        _check(load().tc_reset_kernel_stats(self.handle), "tc_reset_kernel_stats")
