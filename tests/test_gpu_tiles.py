"""Every LDS tile size and workgroup size the autotuner may pick gives the
oracle's counts (integers, tolerance 0): the hub tile (512, 1024, 2048 anchor
entries), the wave and group merge tiles, the group-mode workgroup size and the
batched kernel's tile, each with the dyads or edge records forced into the mode
that uses it, on graphs whose rows are longer than the tiles.  Values outside
the built variants are rejected."""
import functools
import sys
from math import comb

import numpy as np
import pytest

import oracle
from paper_1603_02655_amd import synth, tc

pytestmark = pytest.mark.gpu

BIG = 0xFFFFFFFF
FORCE = {
    "hub": dict(t_hub=0),
    "wave": dict(t0=0, t1=BIG, t_hub=BIG),
    "group": dict(t0=0, t1=0, t_hub=BIG),
}
VARIANTS = (
    [("hub", dict(hub_tile=t)) for t in (512, 1024, 2048)]
    + [("wave", dict(wave_tile=t)) for t in (512, 1024, 2048)]
    + [("group", dict(group_tile=t, group_size=s)) for t in (2048, 4096, 8192) for s in (256, 512)]
)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = tc.Context(0)
    yield c
    c.close()


@functools.lru_cache(maxsize=1)
def _graphs():
    """(n, src, dst, name, oracle census) of the single-graph cases."""
    rng = np.random.default_rng(21)
    # one vertex joined to 5999 others (rows longer than every tile)
    n = 6000
    others = np.arange(1, n, dtype=np.int32)
    out = rng.random(others.size) < 0.5
    src = np.where(out, 0, others).astype(np.int32)
    dst = np.where(out, others, 0).astype(np.int32)
    s2 = rng.integers(0, n, 30000).astype(np.int32)
    d2 = rng.integers(0, n, 30000).astype(np.int32)
    hub = (n, np.concatenate([src, s2]), np.concatenate([dst, d2]), "hub-6000")
    # dense random digraph: forward lists up to n - 1 entries (several hub tiles)
    m = 1300
    mat = rng.random((m, m)) < 0.3
    np.fill_diagonal(mat, False)
    ds, dd = (x.astype(np.int32) for x in np.nonzero(mat))
    dense = (m, ds, dd, "dense-1300")
    g = synth.rmat_digraph(1 << 13, 1 << 17, synth.rng_for(80, 0), reciprocity=0.2)
    return [(n, src, dst, name, oracle.census(n, src, dst).tolist())
            for n, src, dst, name in (hub, dense, (g.n, g.src, g.dst, "rmat-13"))]


@pytest.mark.parametrize("mode,tiles", VARIANTS, ids=[f"{m}-{'-'.join(f'{k}{v}' for k, v in t.items())}"
                                                       for m, t in VARIANTS])
def test_tile_variants_match_oracle(ctx, mode, tiles):
    default = ctx.get_tuning()
    try:
        for n, src, dst, name, want in _graphs():
            for tri in (0, 1):
                ctx.set_tuning(**dict(default, **FORCE[mode], **tiles, tri=tri))
                say(f"[gpu] {name} mode={mode} tiles={tiles} tri={tri}")
                g = ctx.build_graph(n, src, dst)
                try:
                    assert ctx.census(g).tolist() == want, (name, mode, tiles, tri)
                finally:
                    g.release()
    finally:
        ctx.set_tuning(**default)


@functools.lru_cache(maxsize=1)
def _batch_pool():
    """Graphs of the batched cases and their oracle censuses."""
    pool = [synth.batch_graph(i, config=81, n_lo=30, n_hi=5000) for i in range(12)]
    n = 2600
    pool.append(synth.Digraph(n, np.zeros(n - 1, np.int32), np.arange(1, n, dtype=np.int32), "star"))
    rng = np.random.default_rng(82)
    for m, p in ((1100, 1.0), (400, 0.5), (400, 0.15)):     # hub, group and wave records on both paths
        mat = rng.random((m, m)) < p
        np.fill_diagonal(mat, False)
        s, d = (x.astype(np.int32) for x in np.nonzero(mat))
        pool.append(synth.Digraph(m, s, d, f"dense-{m}-{p}"))
    return pool, [oracle.census(g.n, g.src, g.dst).tolist() for g in pool]


@pytest.mark.parametrize("hub_tile", [512, 1024, 2048])
@pytest.mark.parametrize("batch_tile", [512, 1024, 2048])
def test_batch_tiles_match_oracle(ctx, hub_tile, batch_tile):
    pool, want = _batch_pool()
    default = ctx.get_tuning()
    try:
        for tri in (0, 1):
            # thresholds that put dyads in every bucket of the batched kernel
            ctx.set_tuning(**dict(default, t0=16, t1=256, t_hub=1024, hub_tile=hub_tile, batch_tile=batch_tile,
                                  tri=tri))
            say(f"[gpu] batch hub_tile={hub_tile} batch_tile={batch_tile} tri={tri}")
            hs = [ctx.build_graph(g.n, g.src, g.dst) for g in pool]
            try:
                buckets = np.sum([h.info["tri_bucket_edges" if tri else "bucket_dyads"] for h in hs], axis=0)
                assert (buckets > 0).all(), buckets
                assert ctx.census_batch(hs).tolist() == want
                assert ctx.census_batch(hs).tolist() == want          # replay
            finally:
                for h in hs:
                    h.release()
    finally:
        ctx.set_tuning(**default)


def test_unbuilt_tiles_rejected(ctx):
    default = ctx.get_tuning()
    for bad in (dict(hub_tile=768), dict(hub_tile=4096), dict(wave_tile=256), dict(group_tile=1024),
                dict(group_size=128), dict(batch_tile=256)):
        with pytest.raises(tc.TcError) as e:
            ctx.set_tuning(**dict(default, **bad))
        assert e.value.code == tc.TC_ERR_ARG, bad
    assert ctx.get_tuning() == default


def test_complete_digraph_every_hub_tile(ctx):
    n = 2100          # forward lists of up to 2099 entries: more than one 2048-entry tile
    idx = np.arange(n, dtype=np.int32)
    src, dst = np.repeat(idx, n), np.tile(idx, n)
    keep = src != dst
    default = ctx.get_tuning()
    try:
        for hub_tile in (512, 1024, 2048):
            ctx.set_tuning(**dict(default, t_hub=0, hub_tile=hub_tile, tri=1))
            g = ctx.build_graph(n, src[keep], dst[keep])
            try:
                got = ctx.census(g)
                assert int(got[15]) == comb(n, 3) and int(got[1:15].sum()) == 0, hub_tile
            finally:
                g.release()
    finally:
        ctx.set_tuning(**default)
