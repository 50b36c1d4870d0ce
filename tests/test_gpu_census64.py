"""GPU parity of the labelled (64-class) census, tc_census64, against the
oracle's labelled census: bit-exact (tolerance 0) in the default bucket
configuration and with every dyad forced into each execution mode, including
the hub mode, and through the triangles of the forward lists.  The 64-class histogram folded through the class table must also
equal the 16-class census of the same graph."""
import sys
from math import comb

import numpy as np
import pytest

import oracle
from paper_1603_02655_amd import synth, tc
from tests import triads

pytestmark = pytest.mark.gpu

BIG = 0xFFFFFFFF
MODES = {
    "default": None,
    "lane": dict(t0=BIG, t1=BIG, t_hub=BIG, tri=0),
    "wave": dict(t0=0, t1=BIG, t_hub=BIG, tri=0),
    "group": dict(t0=0, t1=0, t_hub=BIG, tri=0),
    "hub": dict(t_hub=0, tri=0),
    "tri": dict(tri=1),
    "tri-lane": dict(t0=BIG, t1=BIG, t_hub=BIG, tri=1),
    "tri-hub": dict(t_hub=0, tri=1),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = tc.Context(0)
    yield c
    c.close()


def fold(c64):
    out = np.zeros(16, np.uint64)
    for k in range(64):
        out[triads.RULE_TABLE[k]] += c64[k]
    return out


def run_modes(ctx, g, want64):
    default = ctx.get_tuning()
    try:
        for mode, tun in MODES.items():
            ctx.set_tuning(**dict(default, **(tun or {})))
            h = ctx.build_graph(g.n, g.src, g.dst)
            try:
                say(f"[gpu] census64 {g.name} n={g.n} m={g.m} mode={mode}")
                got = ctx.census64(h)
                assert got.tolist() == want64.tolist(), (g.name, mode)
                assert fold(got).tolist() == ctx.census(h).tolist(), (g.name, mode)
            finally:
                h.release()
    finally:
        ctx.set_tuning(**default)


@pytest.mark.parametrize("seed", range(6))
def test_random_small(ctx, seed):
    rng = synth.rng_for(640, seed)
    n = int(rng.integers(3, 400))
    m = int(rng.integers(0, 8 * n))
    src = rng.integers(0, n, m).astype(np.int32)
    dst = rng.integers(0, n, m).astype(np.int32)
    g = synth.Digraph(n, src, dst, f"rand{seed}")
    run_modes(ctx, g, oracle.census64(n, src, dst))


def test_stars_and_tiny(ctx):
    n = 3000
    hub = np.arange(1, n, dtype=np.int32)
    for name, s, d in (("out-star-low", np.zeros(n - 1, np.int32), hub),
                       ("in-star-high", hub - 1, np.full(n - 1, n - 1, np.int32))):
        g = synth.Digraph(n, s, d, name)
        run_modes(ctx, g, oracle.census64(n, s, d))
    for n in (0, 1, 2, 3):
        with tc.Context(0) as c:
            h = c.build_graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
            got = c.census64(h)
            assert got[0] == (comb(n, 3) if n >= 3 else 0) and int(got[1:].sum()) == 0
            h.release()


@pytest.mark.parametrize("permute", [True, False])
def test_rmat_medium(ctx, permute):
    g = synth.rmat_digraph(1 << 13, 1 << 17, synth.rng_for(641, int(permute)), reciprocity=0.2,
                           permute=permute)
    run_modes(ctx, g, oracle.census64(g.n, g.src, g.dst))


def test_citation_small(ctx):
    g = synth.citation_dag(40000, 176_000, synth.rng_for(642, 0))
    run_modes(ctx, g, oracle.census64(g.n, g.src, g.dst))
