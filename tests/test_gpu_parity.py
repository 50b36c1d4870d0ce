"""GPU parity: the HIP census through the C ABI against the CPU oracle.

Integer work, so every comparison is bit-exact (tolerance 0).  Each graph is
checked in the default bucket configuration and with every dyad forced into one
execution mode (lane, wave, group, hub), and again through the triangles of the
degree-ordered forward lists with every edge record forced into each mode.  At full workload sizes the whole 16-vector
is compared with the oracle's census stored in tests/golden/ (the graph's arc
hash first), in every path and hub setting; the exact degree identities and the
oracle's task-queue (vertex range) partial census on sampled ranges are checked
too, and the partials of a partition must sum to the full census.
"""
import os
import sys
from math import comb

import numpy as np
import pytest

import oracle
from paper_1603_02655_amd import synth, tc
from tests import triads
from tests.golden import make_goldens as goldens

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
    "tri-wave": dict(t0=0, t1=BIG, t_hub=BIG, tri=1),
    "tri-group": dict(t0=0, t1=0, t_hub=BIG, tri=1),
    "tri-hub": dict(t_hub=0, tri=1),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    oracle.build() if not os.path.exists(oracle.LIB_PATH) else None
    c = tc.Context(0)
    yield c
    c.close()


def gpu_census(ctx, n, src, dst, mode="default"):
    default = ctx.get_tuning()
    try:
        if MODES[mode]:
            ctx.set_tuning(**MODES[mode])
        g = ctx.build_graph(n, src, dst)
        try:
            return ctx.census(g), g.info
        finally:
            g.release()
    finally:
        ctx.set_tuning(**default)


def check(ctx, n, src, dst, want=None, modes=MODES, name=""):
    if want is None:
        want = oracle.census(n, src, dst)
    for mode in modes:
        say(f"[gpu] {name} n={n} m={len(src)} mode={mode}")
        got, info = gpu_census(ctx, n, src, dst, mode)
        assert got.tolist() == want.tolist(), (name, mode, got.tolist(), want.tolist())
        if mode in ("lane", "wave", "group", "hub") and info["bucket_dyads"]:
            idx = {"lane": 0, "wave": 1, "group": 2, "hub": 3}[mode]
            total = sum(info["bucket_dyads"])
            assert info["bucket_dyads"][idx] == total, (mode, info["bucket_dyads"])
        # hub tasks form groups of at most eight consecutive tasks
        for tasks, groups in (("hub_tasks", "hub_groups"), ("tri_tasks", "tri_groups")):
            assert -(-info[tasks] // 8) <= info[groups] <= info[tasks], (mode, info[tasks], info[groups])
        if mode.startswith("tri"):
            assert info["fwd_entries"] == info["asym_dyads"] + info["mutual_dyads"], (mode, info)
            if mode != "tri" and sum(info["tri_bucket_edges"]):
                idx = {"tri-lane": 0, "tri-wave": 1, "tri-group": 2, "tri-hub": 3}[mode]
                assert info["tri_bucket_edges"][idx] == sum(info["tri_bucket_edges"]), (mode, info)
    return want


# ------------------------------------------------------------ small cases ----

def test_paper_example(ctx):
    mat = np.zeros((7, 7), int)
    for a, b in [(0, 1), (0, 2), (0, 3), (3, 4), (3, 5), (4, 4), (5, 3)]:
        mat[a, b] = 1
    src, dst = np.nonzero(mat)
    want = np.array([16, 10, 3, 3, 0, 1, 1, 1, 0, 0, 0, 0, 0, 0, 0, 0], np.uint64)
    check(ctx, 7, src, dst, want, name="paper-7")


@pytest.mark.parametrize("n", [0, 1, 2, 3, 7])
def test_empty_and_tiny(ctx, n):
    check(ctx, n, np.zeros(0, np.int32), np.zeros(0, np.int32), name="empty")


def test_two_vertices(ctx):
    check(ctx, 2, [0, 1], [1, 0], name="n2-mutual")
    check(ctx, 2, [0], [1], name="n2-arc")


@pytest.mark.parametrize("n", [3, 40, 300])
def test_complete_digraph(ctx, n):
    src, dst = np.nonzero(~np.eye(n, dtype=bool))
    want = np.zeros(16, np.uint64)
    want[15] = comb(n, 3)
    check(ctx, n, src, dst, want, name="complete")


def test_cycles_and_stars(ctx):
    n = 1000
    cyc = np.arange(n)
    check(ctx, n, cyc, (cyc + 1) % n, name="cycle")
    check(ctx, n, np.zeros(n - 1, int), np.arange(1, n), name="out-star")
    check(ctx, n, np.arange(1, n), np.zeros(n - 1, int), name="in-star")


def test_tournament(ctx):
    rng = np.random.default_rng(3)
    n = 400
    a, b = np.triu_indices(n, 1)
    flip = rng.random(a.size) < 0.5
    src, dst = np.where(flip, b, a), np.where(flip, a, b)
    check(ctx, n, src, dst, name="tournament")


@pytest.mark.parametrize("seed", range(24))
def test_random_small_vs_oracle(ctx, seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(3, 90))
    mat = rng.random((n, n)) < rng.uniform(0.02, 0.7)
    mat |= mat.T & (rng.random((n, n)) < rng.uniform(0, 1))
    np.fill_diagonal(mat, rng.random(n) < 0.1)
    src, dst = np.nonzero(mat)
    dup = rng.integers(0, max(1, src.size), size=src.size // 4) if src.size else np.zeros(0, int)
    src, dst = np.concatenate([src, src[dup]]), np.concatenate([dst, dst[dup]])
    want = oracle.brute(n, src, dst)
    assert oracle.census(n, src, dst).tolist() == want.tolist()
    check(ctx, n, src, dst, want, name=f"random-{seed}")


# ----------------------------------------------------- adversarial shapes ----

def test_hub_graph(ctx):
    """One vertex joined to everything, plus a sparse random remainder."""
    rng = np.random.default_rng(8)
    n = 6000
    hub = 17
    others = np.array([v for v in range(n) if v != hub])
    out = rng.random(others.size) < 0.5
    src = np.where(out, hub, others)
    dst = np.where(out, others, hub)
    both = rng.random(others.size) < 0.2
    src = np.concatenate([src, others[both]])
    dst = np.concatenate([dst, np.full(both.sum(), hub)])
    s2 = rng.integers(0, n, 20000)
    d2 = rng.integers(0, n, 20000)
    check(ctx, n, np.concatenate([src, s2]), np.concatenate([dst, d2]), name="hub")


def test_dense_mutual_cliques(ctx):
    n = 600
    blocks = np.arange(n) // 150
    mat = (blocks[:, None] == blocks[None, :]) & ~np.eye(n, dtype=bool)
    mat |= np.random.default_rng(1).random((n, n)) < 0.01
    np.fill_diagonal(mat, False)
    src, dst = np.nonzero(mat)
    check(ctx, n, src, dst, name="cliques")


@pytest.mark.parametrize("permute", [True, False])
def test_rmat_medium(ctx, permute):
    g = synth.rmat_digraph(1 << 13, 1 << 17, synth.rng_for(70, int(permute)), reciprocity=0.2, permute=permute)
    check(ctx, g.n, g.src, g.dst, name=f"rmat-13-permute={permute}")


def test_er_config_small(ctx):
    g = synth.config_er_small()
    want = oracle.brute(g.n, g.src, g.dst, threads=min(16, os.cpu_count() or 1))
    check(ctx, g.n, g.src, g.dst, want, name="er-2000")


def test_citation_small(ctx):
    g = synth.citation_dag(200_000, 880_000, synth.rng_for(71, 0))
    check(ctx, g.n, g.src, g.dst, name="citation-200k")


# ----------------------------------------------------------- API behaviour ----

def test_repeat_is_identical(ctx):
    g0 = synth.rmat_digraph(1 << 12, 1 << 16, synth.rng_for(72, 0), reciprocity=0.2)
    g = ctx.build_graph(g0.n, g0.src, g0.dst)
    try:
        a = ctx.census(g)
        for _ in range(5):
            assert ctx.census(g).tolist() == a.tolist()
    finally:
        g.release()


def test_range_partition_sums_to_full(ctx):
    g0 = synth.rmat_digraph(1 << 12, 1 << 16, synth.rng_for(73, 0), reciprocity=0.2)
    g = ctx.build_graph(g0.n, g0.src, g0.dst)
    og = oracle.OracleGraph(g0.n, g0.src, g0.dst)
    try:
        full = ctx.census(g)
        cuts = [0, 1, 100, 2048, 2049, 4000, g0.n]
        parts = np.zeros(16, object)
        for a, b in zip(cuts, cuts[1:]):
            p = ctx.census_range(g, a, b)
            assert p.tolist() == og.census_range(a, b).tolist()
            parts += p.astype(object)
        assert parts[0] == 0
        assert [int(x) for x in parts[1:]] == [int(x) for x in full[1:]]
    finally:
        g.release()
        og.close()


def _sum_shards(ctx, g, nshards):
    parts = [ctx.census_shard(g, k, nshards) for k in range(nshards)]
    for p in parts:
        assert int(p[0]) == 0
    # partials are exact modulo 2^64: add them as uint64, wrapping
    with np.errstate(over="ignore"):
        return np.sum(np.stack(parts).astype(np.uint64), axis=0, dtype=np.uint64)


def test_shards_sum_to_full(ctx):
    g0 = synth.rmat_digraph(1 << 14, 1 << 18, synth.rng_for(74, 0), reciprocity=0.2)
    g = ctx.build_graph(g0.n, g0.src, g0.dst)
    default = ctx.get_tuning()
    try:
        full = ctx.census(g)
        assert triads.identity_violations(g0.n, g0.src, g0.dst, full) == []
        for tri, t_hub in ((1, default["t_hub"]), (1, 0), (0, default["t_hub"]), (0, 0)):
            ctx.set_tuning(**dict(default, tri=tri, t_hub=t_hub))
            ctx.rebucket(g)
            info = g.info
            say(f"[gpu] shards tri={tri} t_hub={t_hub} hub_groups={info['hub_groups']} "
                f"tri_groups={info['tri_groups']}")
            if t_hub == 0:
                assert (info["tri_groups"] if tri else info["hub_groups"]) > 8
            for nshards in (1, 3, 8, 61):
                s = _sum_shards(ctx, g, nshards)
                assert s[1:].tolist() == full[1:].tolist(), (tri, t_hub, nshards)
        for bad in ((0, 0), (-1, 2), (2, 2)):
            with pytest.raises(tc.TcError):
                ctx.census_shard(g, *bad)
    finally:
        ctx.set_tuning(**default)
        ctx.rebucket(g)
        g.release()


def test_info_counts(ctx):
    src = [0, 0, 1, 2, 2, 3, 3]
    dst = [1, 1, 0, 2, 3, 2, 0]
    g = ctx.build_graph(5, src, dst)
    try:
        info = g.info
        assert info["arcs_in"] == 7
        assert info["self_loops_dropped"] == 1
        assert info["duplicates_dropped"] == 1
        assert info["arcs_kept"] == 5
        assert info["mutual_dyads"] == 2 and info["asym_dyads"] == 1
        assert info["max_degree"] == 2
    finally:
        g.release()


def test_errors(ctx):
    with pytest.raises(tc.TcError) as e:
        ctx.build_graph(3, [0, 1], [1, 3])
    assert e.value.code == tc.TC_ERR_ARG
    with pytest.raises(tc.TcError) as e:
        ctx.build_graph(3, [-1], [1])
    assert e.value.code == tc.TC_ERR_ARG
    with pytest.raises(tc.TcError) as e:
        ctx.build_graph(4_801_281, [0], [1])
    assert e.value.code == tc.TC_ERR_RANGE
    with pytest.raises(tc.TcError) as e:
        ctx.build_graph(7, [0, 4], [1, 4], strict=True)
    assert e.value.code == tc.TC_ERR_ARG
    with pytest.raises(tc.TcError) as e:
        ctx.build_graph(7, [0, 0], [1, 1], strict=True)
    assert e.value.code == tc.TC_ERR_ARG
    g = ctx.build_graph(7, [0, 1], [1, 2], strict=True)
    g.release()


def test_max_n_accepted(ctx):
    n = 4_801_280
    g = ctx.build_graph(n, [0, 1, 2], [1, 2, 0])
    try:
        got = ctx.census(g)
        assert int(got[9]) == 1
        assert sum(int(x) for x in got) == comb(n, 3)
        assert int(got[0]) == comb(n, 3) - 1 - 3 * (n - 3)
    finally:
        g.release()


def test_device_pointer_build(ctx):
    g0 = synth.rmat_digraph(1 << 11, 1 << 14, synth.rng_for(74, 0), reciprocity=0.2)
    s = tc.DeviceArray(g0.src)
    d = tc.DeviceArray(g0.dst)
    g = ctx.build_graph(g0.n, s, d)
    s.free()
    d.free()
    try:
        assert ctx.census(g).tolist() == oracle.census(g0.n, g0.src, g0.dst).tolist()
    finally:
        g.release()


# ---------------------------------------------------------- full-size ----

def _ranges_with_work(g0, budget, count, rng):
    """Vertex ranges whose canonical-dyad work sum(|N(u)|+|N(v)|) stays under budget."""
    n = g0.n
    s = g0.src.astype(np.int64)
    d = g0.dst.astype(np.int64)
    keep = s != d
    lo = np.minimum(s[keep], d[keep])
    hi = np.maximum(s[keep], d[keep])
    pk = np.unique(lo * n + hi)
    a, b = pk // n, pk % n
    deg = np.bincount(a, minlength=n) + np.bincount(b, minlength=n)
    work = np.bincount(a, weights=(deg[a] + deg[b]).astype(np.float64), minlength=n)
    cum = np.concatenate([[0.0], np.cumsum(work)])
    out = []
    for _ in range(count):
        u0 = int(rng.integers(0, n))
        u1 = int(np.searchsorted(cum, cum[u0] + budget, side="right")) - 1
        u1 = max(u0 + 1, min(n, u1))
        out.append((u0, u1))
    return out


@pytest.mark.parametrize("which", ["rmat", "citation"])
def test_full_size_identities_and_sampled_ranges(ctx, which):
    say(f"[gpu] generating {which}")
    g0 = synth.config_rmat_2p20() if which == "rmat" else synth.config_citation()
    gold = goldens.load(which)[0]
    assert (g0.n, g0.m, goldens.arc_hash(g0.src, g0.dst)) == (gold["n"], gold["m"], gold["hash"])
    say(f"[gpu] building {which} n={g0.n} m={g0.m}")
    g = ctx.build_graph(g0.n, g0.src, g0.dst)
    og = oracle.OracleGraph(g0.n, g0.src, g0.dst)
    try:
        say(f"[gpu] census {which}")
        full = ctx.census(g)
        # the whole 16-vector against the oracle's census of the same graph
        assert [int(x) for x in full] == gold["counts"]
        assert triads.identity_violations(g0.n, g0.src, g0.dst, full) == []
        assert ctx.census(g).tolist() == full.tolist()
        # R-MAT's forward-list hub bucket holds more than 2^20 edges, so it has
        # both hub task sets: the half-size one ran in the census above, and a
        # batched launch runs the full-size one
        assert g.info["tri_chunk"] == (256 if which == "rmat" else 512)
        say(f"[gpu] batched census of {which} alone")
        assert ctx.census_batch([g])[0].tolist() == full.tolist()
        say(f"[gpu] shards {which}")
        assert _sum_shards(ctx, g, 8)[1:].tolist() == full[1:].tolist()
        rng = np.random.default_rng(5)
        for u0, u1 in _ranges_with_work(g0, 2e7, 3, rng):
            say(f"[gpu] range {which} [{u0},{u1})")
            assert ctx.census_range(g, u0, u1).tolist() == og.census_range(u0, u1).tolist()
        # through the dyad records, with every dyad in the hub mode, and with none
        default = ctx.get_tuning()
        for t_hub in (0, BIG):
            ctx.set_tuning(t_hub=t_hub, tri=0)
            ctx.rebucket(g)
            say(f"[gpu] {which} t_hub={t_hub} buckets={g.info['bucket_dyads']}")
            assert ctx.census(g).tolist() == full.tolist()
            u0, u1 = _ranges_with_work(g0, 2e7, 1, rng)[0]
            assert ctx.census_range(g, u0, u1).tolist() == og.census_range(u0, u1).tolist()
        # through the triangles of the forward lists, default and all-hub buckets
        for t_hub in (BIG, 0):
            ctx.set_tuning(**dict(default, t_hub=t_hub, tri=1))
            ctx.rebucket(g)
            say(f"[gpu] {which} tri t_hub={t_hub} edges={g.info['tri_bucket_edges']}")
            assert ctx.census(g).tolist() == full.tolist()
        ctx.set_tuning(**default)
    finally:
        ctx.set_tuning(**default)
        g.release()
        og.close()


# ------------------------------------------- forward lists longer than a tile ----

def _modes_agree(ctx, n, src, dst, modes):
    out = {}
    for mode in modes:
        say(f"[gpu] long forward lists n={n} m={len(src)} mode={mode}")
        got, info = gpu_census(ctx, n, src, dst, mode)
        out[mode] = got
    first = next(iter(out.values()))
    for mode, got in out.items():
        assert got.tolist() == first.tolist(), mode
    return first


def test_forward_lists_longer_than_a_tile(ctx):
    # degree ties are broken by id, so in a complete digraph N+(x) holds the
    # n - 1 - x vertices above x: the first vertices' forward lists span two
    # LDS tiles of the hub mode (1024 entries)
    n = 1100
    idx = np.arange(n, dtype=np.int32)
    src = np.repeat(idx, n)
    dst = np.tile(idx, n)
    keep = src != dst
    got = _modes_agree(ctx, n, src[keep], dst[keep], ["default", "tri-hub", "hub"])
    want = np.zeros(16, np.uint64)
    want[triads.INDEX["300"]] = comb(n, 3)
    assert got.tolist() == want.tolist()
    # random tournament: 030T = sum over v of C(out(v), 2), the rest 030C
    rng = np.random.default_rng(1100)
    a, b = np.triu_indices(n, 1)
    flip = rng.random(a.size) < 0.5
    s, d = np.where(flip, b, a).astype(np.int32), np.where(flip, a, b).astype(np.int32)
    got = _modes_agree(ctx, n, s, d, ["default", "tri-hub", "hub", "group"])
    outdeg = np.bincount(s, minlength=n)
    t030 = sum(comb(int(k), 2) for k in outdeg)
    want = np.zeros(16, np.uint64)
    want[triads.INDEX["030T"]] = t030
    want[triads.INDEX["030C"]] = comb(n, 3) - t030
    assert got.tolist() == want.tolist()


def test_dense_digraph_identities_across_modes(ctx):
    n = 1100
    rng = np.random.default_rng(1101)
    mat = rng.random((n, n)) < 0.75
    np.fill_diagonal(mat, False)
    src, dst = (x.astype(np.int32) for x in np.nonzero(mat))
    got = _modes_agree(ctx, n, src, dst, ["default", "tri-hub", "tri-lane", "hub", "lane"])
    assert triads.identity_violations(n, src, dst, got) == []
