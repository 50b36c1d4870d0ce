"""The stored full-size census goldens (tests/golden/census_*.txt, written by
tests/golden/make_goldens.py from the CPU oracle) checked on the CPU:

* every row sums to C(n, 3) (section "Triad Census Algorithm": the 16 classes
  partition the triples);
* the exact degree identities (sum, dyad-type counts times n - 2, wedges,
  out- and in-pairs, two-paths) hold for the regenerated R-MAT 2^20 and
  citation graphs, and for a sample of the pool graphs;
* a seeded sample of the pool graphs, including the largest batch graph, is
  regenerated (same arc hash) and its census recomputed by the oracle.

Set TC_REGEN_GOLDENS=1 to also recompute the R-MAT 2^20 vector with the
multithreaded oracle (a few minutes).
"""
import os
from math import comb

import numpy as np
import pytest

import oracle
from tests import triads
from tests.golden import make_goldens as goldens


@pytest.mark.parametrize("kind", sorted(goldens.FILES))
def test_rows_sum_to_triples(kind):
    rows = goldens.load(kind)
    assert rows
    for r in rows:
        assert sum(r["counts"]) == comb(r["n"], 3), r["name"]
        assert all(c >= 0 for c in r["counts"])


def test_pool_sizes():
    assert len(goldens.load("batch")) == goldens.BATCH_COUNT
    assert len(goldens.load("serve")) == goldens.SERVE_COUNT
    assert [r["name"] for r in goldens.load("batch")] == [f"batch-{i}" for i in range(goldens.BATCH_COUNT)]


def _sample(kind, count, seed, max_arcs):
    rows = goldens.load(kind)
    rng = np.random.default_rng(seed)
    idx = [int(i) for i in rng.permutation(len(rows)) if rows[i]["m"] <= max_arcs][:count]
    if kind == "batch":
        idx.append(max(range(len(rows)), key=lambda i: rows[i]["n"]))   # the largest graph
    return [(i, rows[i]) for i in idx]


@pytest.mark.parametrize("kind,count,max_arcs", [("batch", 24, 10**9), ("serve", 8, 400_000)])
def test_pool_sample_regenerated(kind, count, max_arcs):
    for i, rec in _sample(kind, count, 7, max_arcs):
        g, h = goldens.graph_with_hash((kind, i))
        assert (g.n, g.m, h) == (rec["n"], rec["m"], rec["hash"]), rec["name"]
        assert [int(x) for x in oracle.census(g.n, g.src, g.dst)] == rec["counts"], rec["name"]
        assert triads.identity_violations(g.n, g.src, g.dst, np.array(rec["counts"], dtype=object)) == []


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["rmat", "citation"])
def test_full_graph_identities(kind):
    rec = goldens.load(kind)[0]
    g, h = goldens.graph_with_hash((kind, 0))
    assert (g.n, g.m, h) == (rec["n"], rec["m"], rec["hash"])
    assert triads.identity_violations(g.n, g.src, g.dst, np.array(rec["counts"], dtype=object)) == []
    if kind == "rmat" and os.environ.get("TC_REGEN_GOLDENS") == "1":
        with oracle.OracleGraph(g.n, g.src, g.dst) as og:
            assert [int(x) for x in og.census_mt(os.cpu_count() or 1)] == rec["counts"]
