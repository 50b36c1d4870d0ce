"""Planted mistakes in copies of the oracle must be caught by the pins.

Each mutant is a text edit of oracle.c (a dropped condition, an off-by-one, a
transposed operand, a stale look-up, ...) compiled into a temporary library on
the CPU.  The
test asserts that at least one independent pin (rule-based Python brute force,
the thesis's worked example, the degree identities) rejects it.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

from tests import triads

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "oracle.c")

MUTANTS = {
    "third-vertex-joined-to-x": ("if (q <= x || ws->in_x[q] == (int64_t)x + 1) continue;",
                                 "if (q <= x) continue;"),
    "third-vertex-may-be-x": ("if (q <= x || ws->in_x[q] == (int64_t)x + 1) continue;",
                              "if (q < x || ws->in_x[q] == (int64_t)x + 1) continue;"),
    "pair-q-equal-p": ("if (q <= p) continue;", "if (q < p) continue;"),
    "both-orientations": ("if (p < x) continue;\n", "\n"),
    "single-pair-off-by-one": ("(uint64_t)(n - 2 - touched)", "(uint64_t)(n - 1 - touched)"),
    "touched-counts-x": ("if (w != x && ws->in_x[w] != (int64_t)x + 1) ++touched;",
                         "if (ws->in_x[w] != (int64_t)x + 1) ++touched;"),
    "stale-p-table": ("ws->in_p[q] == key ? ws->dir_p[q] : 0", "ws->dir_p[q]"),
    "direction-transposed": ("arc(g, x, w) | (arc(g, w, x) << 1)", "arc(g, w, x) | (arc(g, x, w) << 1)"),
    "null-count": ("(u128)(n - 2) / 6", "(u128)(n - 3) / 6"),
    "no-neighbour-dedup": ("if (i == 0 || ukey[i] != ukey[i - 1]) ukey[b++] = ukey[i];",
                           "ukey[b++] = ukey[i];"),
    "swap-111-labels": ("/* 111D */ {0, 1, 1, 0, 2, 1, -1},", "/* 111D */ {0, 1, 1, 0, 1, 2, -1},"),
}


def _build_mutant(name, tmpdir):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutation anchor missing: {old}"
    text = text.replace(old, new)
    if name == "swap-111-labels":
        text = text.replace("/* 111U */ {0, 1, 1, 0, 1, 2, -1},", "/* 111U */ {0, 1, 1, 0, 2, 1, -1},")
    c = os.path.join(tmpdir, f"{name}.c")
    so = os.path.join(tmpdir, f"{name}.so")
    with open(c, "w") as f:
        f.write(text)
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-fPIC", "-shared", "-pthread", c, "-o", so],
                   check=True)
    lib = ctypes.CDLL(so)
    lib.oracle_graph_new.restype = ctypes.c_void_p
    lib.oracle_graph_new.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_census.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.oracle_graph_free.argtypes = [ctypes.c_void_p]
    return lib


def _census(lib, n, src, dst):
    s = np.ascontiguousarray(src, np.int32)
    d = np.ascontiguousarray(dst, np.int32)
    h = lib.oracle_graph_new(n, s.size, s.ctypes.data, d.ctypes.data)
    if not h:
        return None
    out = np.zeros(16, np.uint64)
    lib.oracle_census(h, out.ctypes.data)
    lib.oracle_graph_free(h)
    return out


def _pins_reject(lib):
    rng = np.random.default_rng(77)
    for _ in range(30):
        n = int(rng.integers(3, 10))
        mat = rng.random((n, n)) < rng.uniform(0.1, 0.9)
        np.fill_diagonal(mat, False)
        src, dst = np.nonzero(mat)
        src = np.concatenate([src, src[: len(src) // 3]])
        dst = np.concatenate([dst, dst[: len(dst) // 3]])
        got = _census(lib, n, src, dst)
        if got is None or got.tolist() != triads.brute_census(n, src, dst).tolist():
            return True
        if triads.identity_violations(n, src, dst, got):
            return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name):
    with tempfile.TemporaryDirectory() as tmp:
        lib = _build_mutant(name, tmp)
        assert _pins_reject(lib), f"mutant {name} survived the pins"


# Mistakes planted only in the labelled (64-class) census body: its classes
# are unchanged by most of them, so the brute force by triples must catch them.
MUTANTS64 = {
    "dyadic-term-to-null": ("hist[uv] += (uint64_t)(n - 2 - touched);",
                            "hist[0] += (uint64_t)(n - 2 - touched);"),
    "uv-pair-transposed": ("const int uv = ws->dir_x[p];",
                           "const int uv = (ws->dir_x[p] >> 1) | ((ws->dir_x[p] & 1) << 1);"),
    "u-and-v-roles-swapped": ("hist[uv | ws->dir_p[q] << 4] += 1;",
                              "hist[(uv >> 1 | (uv & 1) << 1) | ws->dir_p[q] << 2] += 1;"),
}


def _census64(lib, n, src, dst):
    s = np.ascontiguousarray(src, np.int32)
    d = np.ascontiguousarray(dst, np.int32)
    h = lib.oracle_graph_new(n, s.size, s.ctypes.data, d.ctypes.data)
    out = np.zeros(64, np.uint64)
    lib.oracle_census64(h, out.ctypes.data)
    lib.oracle_graph_free(h)
    return out


@pytest.mark.parametrize("name", sorted(MUTANTS64))
def test_census64_pins_catch_mutant(name):
    old, new = MUTANTS64[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor missing or ambiguous: {name}"
    with tempfile.TemporaryDirectory() as tmp:
        c, so = os.path.join(tmp, "m.c"), os.path.join(tmp, "m.so")
        with open(c, "w") as f:
            f.write(text.replace(old, new))
        subprocess.run(["gcc", "-O1", "-std=gnu11", "-fPIC", "-shared", "-pthread", c, "-o", so], check=True)
        lib = ctypes.CDLL(so)
        lib.oracle_graph_new.restype = ctypes.c_void_p
        lib.oracle_graph_new.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_census64.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        lib.oracle_graph_free.argtypes = [ctypes.c_void_p]
        rng = np.random.default_rng(78)
        caught = False
        for _ in range(20):
            n = int(rng.integers(3, 10))
            mat = rng.random((n, n)) < rng.uniform(0.1, 0.9)
            np.fill_diagonal(mat, False)
            src, dst = np.nonzero(mat)
            if _census64(lib, n, src, dst).tolist() != triads.brute_census64(n, src, dst).tolist():
                caught = True
                break
        assert caught, f"mutant {name} survived the pins"
