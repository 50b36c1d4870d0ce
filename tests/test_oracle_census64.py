"""Pins of the oracle's 64-class labelled census (the raw TriadCode
histogram of the section on TriadCode, before the table folds it into 16
classes).  The labelled census depends on which vertex plays u, v and w, so
it has no relabelling invariance; it is pinned by a triple-by-triple brute
force whose roles come from the loop's counting condition, by closed forms
for stars whose centre is the smallest or the largest id, by the transpose
(which swaps the two bits of every pair), and by its projection through the
table onto the (separately pinned) 16-class census."""
from math import comb

import numpy as np
import pytest

import oracle
from paper_1603_02655_amd import synth
from tests import triads


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def swap_pairs(code: int) -> int:
    """Transposing every arc swaps bits (1,2), (4,8) and (16,32)."""
    return triads.transpose(code)


def project(c64):
    out = np.zeros(16, np.uint64)
    for k in range(64):
        out[triads.RULE_TABLE[k]] += c64[k]
    return out


def test_brute_force_tiny_random():
    rng = np.random.default_rng(64)
    for trial in range(30):
        n = int(rng.integers(3, 14))
        m = int(rng.integers(0, n * 3))
        src = rng.integers(0, n, m)
        dst = rng.integers(0, n, m)
        got = oracle.census64(n, src, dst)
        assert got.tolist() == triads.brute_census64(n, src, dst).tolist(), trial


def test_out_star_centre_smallest():
    # arcs 0 -> k: every triple {0, j, k} is counted from dyad (0, j) with
    # w = k: u->v and u->w, code 1 + 4
    n = 9
    got = oracle.census64(n, [0] * (n - 1), list(range(1, n)))
    want = np.zeros(64, np.uint64)
    want[5] = comb(n - 1, 2)
    want[0] = comb(n - 1, 3)
    assert got.tolist() == want.tolist()


def test_out_star_centre_largest():
    # arcs (n-1) -> k: triple {j, k, n-1} is counted from dyad (j, n-1) with
    # w = k: v->u and v->w, code 2 + 16
    n = 9
    got = oracle.census64(n, [n - 1] * (n - 1), list(range(n - 1)))
    want = np.zeros(64, np.uint64)
    want[18] = comb(n - 1, 2)
    want[0] = comb(n - 1, 3)
    assert got.tolist() == want.tolist()


def test_single_arc_and_mutual_pair():
    n = 7
    a = oracle.census64(n, [4], [2])          # dyad (2, 4) with v -> u
    assert a[2] == n - 2 and a[0] == comb(n, 3) - (n - 2) and a.sum() == comb(n, 3)
    b = oracle.census64(n, [1, 3], [3, 1])
    assert b[3] == n - 2 and b[0] == comb(n, 3) - (n - 2)


def test_transpose_swaps_bit_pairs():
    g = synth.rmat_digraph(600, 4000, synth.rng_for(64, 1), reciprocity=0.15)
    a = oracle.census64(g.n, g.src, g.dst)
    b = oracle.census64(g.n, g.dst, g.src)
    assert [int(b[swap_pairs(k)]) for k in range(64)] == a.tolist()


def test_projection_is_the_census_and_no_code_lacks_the_dyad():
    for seed in range(3):
        g = synth.rmat_digraph(1500, 12000, synth.rng_for(64, 10 + seed), reciprocity=0.2)
        c64 = oracle.census64(g.n, g.src, g.dst)
        assert project(c64).tolist() == oracle.census(g.n, g.src, g.dst).tolist()
        # the (u, v) pair of a counted triple is always joined
        assert all(c64[k] == 0 for k in range(4, 64, 4))
        assert int(c64.sum()) == comb(g.n, 3)


def test_relabelling_changes_labels_not_classes():
    g = synth.rmat_digraph(400, 3000, synth.rng_for(64, 20), reciprocity=0.1)
    h = synth.relabel(g, synth.rng_for(64, 21))
    a, b = oracle.census64(g.n, g.src, g.dst), oracle.census64(h.n, h.src, h.dst)
    assert project(a).tolist() == project(b).tolist()
    assert a.tolist() != b.tolist()
