"""Seeded synthetic digraphs shaped like the workloads of the triad-census study.

This module only draws random directed graphs (arrays of arc tails and heads)
and reports their shape statistics.  It contains none of the census arithmetic
and is the one piece of code shared by the CPU oracle tests and the GPU path.

The thesis measured real social/citation networks (Actors, Patents, Amazon,
Slashdot, Google; section "Data sets" of the experimental chapter) that are not
available here.  These generators stand in for them with seeded random graphs
of the same order, size and degree-skew shape:

* ``er_digraph``      Erdos-Renyi G(n, p) over ordered pairs.
* ``rmat_digraph``    R-MAT (recursive quadrant) arcs with a prescribed
                      reciprocity, duplicates and self-loops removed.
* ``citation_dag``    arcs from higher to lower ids, lognormal out-degree and a
                      copy model for heads (heavy in-degree tail), sized like
                      the Patents citation graph (3.77 M vertices, 16.5 M arcs,
                      aggregate neighbour-set size of about 7.05e8 in the
                      load-balance comparison table).
* ``batch_pool`` / ``serving_pool``  many uneven graphs for batched / served runs.

Every generator takes an explicit ``numpy.random.Generator``; ``rng_for``
derives independent streams from a base seed with SplitMix64 so that graph
``i`` of configuration ``k`` is reproducible on its own.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BASE_SEED = 0x16030265
_MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """One step of SplitMix64 (Steele, Lea, Flood 2014) on a Python int."""
    x = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = x
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def rng_for(config: int, index: int = 0, base: int = BASE_SEED) -> np.random.Generator:
    """Independent PCG64 stream for graph ``index`` of configuration ``config``."""
    s = splitmix64((base + config) & _MASK64)
    s = splitmix64(s ^ ((index * 0xD1B54A32D192ED03) & _MASK64))
    return np.random.Generator(np.random.PCG64(s))


@dataclass
class Digraph:
    """A directed graph as arc arrays (int32 tails/heads, 0-based ids)."""
    n: int
    src: np.ndarray
    dst: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


# --------------------------------------------------------------------------
# helpers on arc sets (no census arithmetic)
# --------------------------------------------------------------------------

def _keys(src: np.ndarray, dst: np.ndarray, n: int) -> np.ndarray:
    return src.astype(np.int64) * np.int64(n) + dst.astype(np.int64)


def _unique_arcs(src, dst, n):
    keep = src != dst
    k = np.unique(_keys(src[keep], dst[keep], n))
    return (k // n).astype(np.int32), (k % n).astype(np.int32)


def relabel(g: Digraph, rng: np.random.Generator) -> Digraph:
    """Apply a uniformly random vertex permutation and shuffle the arc order."""
    perm = rng.permutation(g.n).astype(np.int32)
    order = rng.permutation(g.m)
    return Digraph(g.n, perm[g.src][order], perm[g.dst][order], g.name)


def add_reciprocity(src, dst, n, target_r, rng):
    """Add reverses of randomly chosen one-way arcs until the fraction of arcs
    whose reverse is present reaches ``target_r`` (never above it)."""
    k = _keys(src, dst, n)
    rk = _keys(dst, src, n)
    ks = np.sort(k)
    pos = np.searchsorted(ks, rk)
    pos[pos >= ks.size] = 0
    has_rev = ks[pos] == rk
    m = src.size
    mutual_arcs = int(has_rev.sum())
    # after adding x reverses: (mutual_arcs + 2x) / (m + x) = r
    x = int(round((target_r * m - mutual_arcs) / (2.0 - target_r)))
    one_way = np.flatnonzero(~has_rev)
    if x <= 0 or one_way.size == 0:
        return src, dst
    x = min(x, one_way.size)
    pick = rng.choice(one_way, size=x, replace=False)
    return (np.concatenate([src, dst[pick]]).astype(np.int32),
            np.concatenate([dst, src[pick]]).astype(np.int32))


# --------------------------------------------------------------------------
# generators
# --------------------------------------------------------------------------

def er_digraph(n: int, p: float, rng: np.random.Generator, name: str = "er") -> Digraph:
    """G(n, p) on ordered pairs u != v: every possible arc independently with
    probability p.  The arc count is drawn from its binomial law and that many
    distinct ordered pairs are then drawn uniformly, which is the same law."""
    pairs = n * (n - 1)
    if pairs == 0 or p <= 0.0:
        return Digraph(n, np.zeros(0, np.int32), np.zeros(0, np.int32), name)
    m = int(rng.binomial(pairs, p))
    if pairs <= 4_000_000:
        idx = np.sort(rng.choice(pairs, size=m, replace=False))
    else:
        idx = np.zeros(0, np.int64)
        while idx.size < m:
            more = rng.integers(0, pairs, size=int((m - idx.size) * 1.05) + 16)
            idx = np.unique(np.concatenate([idx, more]))
        idx = rng.permutation(idx)[:m]
    u = idx // (n - 1)
    r = idx % (n - 1)
    v = r + (r >= u)  # skip the diagonal
    order = rng.permutation(m)
    return Digraph(n, u[order].astype(np.int32), v[order].astype(np.int32), name)


def _rmat_draw(count, scale, abcd, rng):
    a, b, c, _ = abcd
    src = np.zeros(count, np.int64)
    dst = np.zeros(count, np.int64)
    t1, t2, t3 = np.float32(a), np.float32(a + b), np.float32(a + b + c)
    for _ in range(scale):
        r = rng.random(count, dtype=np.float32)
        bi = r >= t2
        bj = ((r >= t1) & (r < t2)) | (r >= t3)
        src = (src << 1) | bi
        dst = (dst << 1) | bj
    return src, dst


def rmat_digraph(n: int, m_target: int, rng: np.random.Generator,
                 abcd=(0.57, 0.19, 0.19, 0.05), reciprocity: float = 0.0,
                 permute: bool = True, name: str = "rmat") -> Digraph:
    """R-MAT arcs at scale ceil(log2 n) (ids >= n rejected), self-loops and
    duplicates dropped, then reverses of one-way arcs added so that the
    reciprocity reaches ``reciprocity``; the total lands near ``m_target``."""
    scale = max(1, math.ceil(math.log2(max(n, 2))))
    max_arcs = n * (n - 1)
    m_target = int(min(m_target, max_arcs))
    # base arcs needed so that base + added reverses ~= m_target
    base_need = int(round(m_target / (1.0 + reciprocity / (2.0 - reciprocity))))
    base_need = max(0, min(base_need, max_arcs))
    keys = np.zeros(0, np.int64)
    draw = max(64, int(base_need * 1.15))
    for _ in range(64):
        if keys.size >= base_need:
            break
        s, d = _rmat_draw(draw, scale, abcd, rng)
        ok = (s < n) & (d < n) & (s != d)
        keys = np.unique(np.concatenate([keys, s[ok] * n + d[ok]]))
        draw = max(64, int((base_need - keys.size) * 1.6) + 64)
    keys = rng.permutation(keys)[:base_need]
    src = (keys // n).astype(np.int32)
    dst = (keys % n).astype(np.int32)
    if reciprocity > 0:
        src, dst = add_reciprocity(src, dst, n, reciprocity, rng)
    g = Digraph(n, src, dst, name)
    if permute:
        g = relabel(g, rng)
    return g


def citation_dag(n: int, m_target: int, rng: np.random.Generator,
                 sigma: float = 1.2, max_out: int = 800, copy_prob: float = 0.28,
                 reciprocity: float = 0.005, permute: bool = True,
                 name: str = "citation") -> Digraph:
    """Citation-shaped graph: vertex u cites round(lognormal) lower ids (mean
    out-degree about m_target/n, clipped at ``max_out`` and at u).  Each head is,
    with probability 1 - copy_prob, uniform in [0, u); otherwise it copies the
    head of a uniformly chosen arc of an earlier vertex (copy model, which
    gives the heavy in-degree tail of citation networks).  Duplicates are
    dropped and a small fraction of arcs is reciprocated."""
    mean = m_target / n
    mu = math.log(mean) - sigma * sigma / 2.0
    deg = np.rint(rng.lognormal(mu, sigma, size=n)).astype(np.int64)
    deg = np.minimum(deg, max_out)
    deg = np.minimum(deg, np.arange(n, dtype=np.int64))
    tail = np.repeat(np.arange(n, dtype=np.int64), deg)
    m0 = tail.size
    first = np.zeros(n + 1, np.int64)
    np.cumsum(deg, out=first[1:])
    start_of_tail = first[tail]  # arcs of earlier vertices are [0, start)
    coin = rng.random(m0) < copy_prob
    coin &= start_of_tail > 0
    head = np.floor(rng.random(m0) * tail).astype(np.int64)
    ptr = np.arange(m0, dtype=np.int64)
    j = np.floor(rng.random(m0) * start_of_tail).astype(np.int64)
    ptr[coin] = j[coin]
    # pointer jumping: every copy chain ends at an arc with a uniform head
    for _ in range(64):
        nxt = ptr[ptr]
        if np.array_equal(nxt, ptr):
            break
        ptr = nxt
    head = head[ptr]
    src, dst = _unique_arcs(tail.astype(np.int32), head.astype(np.int32), n)
    if reciprocity > 0:
        src, dst = add_reciprocity(src, dst, n, reciprocity, rng)
    g = Digraph(n, src, dst, name)
    if permute:
        g = relabel(g, rng)
    return g


# --------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------

def config_er_small(seed_index: int = 0) -> Digraph:
    """ER digraph, n = 2000, p = 0.0025 per ordered pair (about 10 k arcs)."""
    return er_digraph(2000, 0.0025, rng_for(1, seed_index), name="er-2000")


def config_rmat_2p20(seed_index: int = 0, permute: bool = True) -> Digraph:
    """R-MAT (0.57, 0.19, 0.19, 0.05), n = 2^20, 2^24 arcs, reciprocity 0.20."""
    return rmat_digraph(1 << 20, 1 << 24, rng_for(2, seed_index), reciprocity=0.20,
                        permute=permute, name="rmat-2^20-16M-r0.2")


def config_citation(seed_index: int = 0) -> Digraph:
    """Citation-shaped DAG, n = 3.8 M, about 16.5 M arcs, reciprocity 0.5 %."""
    return citation_dag(3_800_000, 16_500_000, rng_for(3, seed_index),
                        name="citation-3.8M-16.5M")


def batch_graph(i: int, config: int = 4, n_lo: int = 50, n_hi: int = 20000,
                k_lo: float = 3.0, k_hi: float = 30.0) -> Digraph:
    """Graph ``i`` of the batch pool: n log-uniform in [n_lo, n_hi], mean
    out-degree uniform in [k_lo, k_hi], R-MAT arcs, reciprocity 0.10."""
    rng = rng_for(config, i)
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    k = rng.uniform(k_lo, k_hi)
    m = int(min(round(n * k), 0.5 * n * (n - 1)))
    return rmat_digraph(n, m, rng, reciprocity=0.10, name=f"batch-{i}")


def batch_pool(count: int = 4096, **kw) -> list:
    return [batch_graph(i, **kw) for i in range(count)]


def serving_graph(i: int, config: int = 5, n_lo: int = 1000, n_hi: int = 1_000_000,
                  k_lo: float = 4.0, k_hi: float = 32.0) -> Digraph:
    """Graph ``i`` of the serving pool: even i ER, odd i R-MAT (reciprocity
    0.10); n log-uniform in [n_lo, n_hi]; mean out-degree uniform in [k_lo, k_hi]."""
    rng = rng_for(config, i)
    n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
    k = rng.uniform(k_lo, k_hi)
    if i % 2 == 0:
        return er_digraph(n, min(1.0, k / max(n - 1, 1)), rng, name=f"serve-er-{i}")
    m = int(min(round(n * k), 0.5 * n * (n - 1)))
    return rmat_digraph(n, m, rng, reciprocity=0.10, name=f"serve-rmat-{i}")


def poisson_arrivals(rate: float, duration: float, rng: np.random.Generator) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    out = []
    t = 0.0
    while True:
        gaps = rng.exponential(1.0 / rate, size=max(16, int(rate * duration * 0.2) + 16))
        ts = t + np.cumsum(gaps)
        keep = ts[ts < duration]
        out.append(keep)
        if keep.size < ts.size:
            break
        t = ts[-1]
    return np.concatenate(out)


# --------------------------------------------------------------------------
# shape statistics (workload shape only)
# --------------------------------------------------------------------------

def shape_stats(g: Digraph) -> dict:
    """Order, size after canonicalisation, reciprocity, undirected degrees.

    ``sum_d2`` is the sum over vertices of |N(u)|^2 with N(u) the undirected
    neighbourhood; it equals the aggregate |N(u)|+|N(v)| over connected pairs,
    which is the cost measure of the canonical-dyad load balance."""
    n = g.n
    keep = g.src != g.dst
    s = g.src[keep].astype(np.int64)
    d = g.dst[keep].astype(np.int64)
    k = np.unique(s * n + d)
    s, d = k // n, k % n
    lo = np.minimum(s, d)
    hi = np.maximum(s, d)
    pk, cnt = np.unique(lo * n + hi, return_counts=True)
    a, b = pk // n, pk % n
    deg = np.bincount(a, minlength=n) + np.bincount(b, minlength=n)
    m = int(k.size)
    mutual_pairs = int((cnt == 2).sum())
    return dict(n=n, m=m, pairs=int(pk.size), mutual_pairs=mutual_pairs,
                reciprocity=(2.0 * mutual_pairs / m) if m else 0.0,
                sum_d2=int((deg.astype(np.int64) ** 2).sum()),
                max_degree=int(deg.max()) if n else 0)
