"""Full-vector parity over the batch and serving pools at their full sizes:
the GPU census, through the C ABI, against the oracle's 16-class census stored
in tests/golden/ (written by tests/golden/make_goldens.py from the CPU oracle
only; the R-MAT 2^20 and citation vectors are compared in test_gpu_parity).  Each graph is
regenerated from its seed and its arc hash is compared with the stored one
before any count is.  Integer counts: tolerance 0.

* the batch pool, all 4096 graphs, in one persistent batched launch (default
  tuning and per-dyad records), replayed;
* the first 64 graphs of the serving pool, requested in a random mix through
  the serving loop (continuous batching).
"""
import multiprocessing as mp
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from paper_1603_02655_amd import tc
from tests.golden import make_goldens as goldens

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = tc.Context(0)
    yield c
    c.close()


def generate(kind, count):
    """Pool graphs 0..count-1 with their arc hashes, drawn in spawned worker
    processes (which never touch the GPU)."""
    workers = max(1, min(16, os.cpu_count() or 1))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        jobs = [(kind, i) for i in range(count)]
        return list(ex.map(goldens.graph_with_hash, jobs, chunksize=max(1, count // (4 * workers))))


def check_hashes(pool, gold):
    assert len(pool) == len(gold)
    for (g, h), rec in zip(pool, gold):
        assert (g.n, g.m, h) == (rec["n"], rec["m"], rec["hash"]), (rec["name"], g.n, g.m, h)


def test_batch_pool_vs_golden(ctx):
    gold = goldens.load("batch")
    say(f"[gpu] generating {len(gold)} batch graphs")
    pool = generate("batch", len(gold))
    check_hashes(pool, gold)
    want = np.array([r["counts"] for r in gold], dtype=np.uint64)
    say("[gpu] building the batch pool")
    handles = [ctx.build_graph(g.n, g.src, g.dst) for g, _ in pool]
    default = ctx.get_tuning()
    try:
        for tuning in (None, dict(tri=0)):
            if tuning:
                ctx.set_tuning(**dict(default, **tuning))
                for h in handles:
                    ctx.rebucket(h)
            say(f"[gpu] batched census of {len(handles)} graphs, tuning {tuning or 'default'}")
            got = ctx.census_batch(handles)
            bad = [gold[i]["name"] for i in range(len(gold)) if got[i].tolist() != want[i].tolist()]
            assert not bad, bad[:10]
            again = ctx.census_batch(handles)            # replay of the captured launch
            assert again.tolist() == want.tolist()
    finally:
        ctx.set_tuning(**default)
        for h in handles:
            h.release()


def test_serving_pool_vs_golden():
    gold = goldens.load("serve")
    say(f"[gpu] generating {len(gold)} serving graphs")
    pool = generate("serve", len(gold))
    check_hashes(pool, gold)
    with tc.Context(0) as c:
        handles = [c.build_graph(g.n, g.src, g.dst) for g, _ in pool]
        rng = np.random.default_rng(11)
        order = rng.integers(0, len(handles), 400)
        say(f"[gpu] serving {order.size} requests over {len(handles)} resident graphs")
        tickets = []
        for k, i in enumerate(order):
            tickets.append((c.submit(handles[i]), int(i)))
            if k % 25 == 0:
                time.sleep(0.001)          # arrivals spread out: many rounds, mixed sizes
        done = {}
        t0 = time.time()
        while len(done) < len(tickets):
            for t, _ in tickets:
                if t not in done:
                    r = c.poll(t)
                    if r is not None:
                        done[t] = r
            assert time.time() - t0 < 120, "serving did not finish"
        for t, i in tickets:
            assert [int(x) for x in done[t]] == gold[i]["counts"], gold[i]["name"]
        st = c.serve_stats()
        say(f"[gpu] serve stats {st}")
        assert st["rounds"] >= 2
        for h in handles:
            h.release()
