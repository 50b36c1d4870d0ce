"""tc_census_each_noalloc (no device allocation; scratch in a fixed device
array of the library) against tc_census_each on the same resident graphs:
identical counts (integers, tolerance 0) on two calls in a row, the second with
fewer and smaller graphs, and the size limit."""
import sys

import numpy as np
import pytest

import oracle
from paper_1603_02655_amd import synth, tc

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pool():
    gs = [synth.batch_graph(i, config=60, n_lo=30, n_hi=6000) for i in range(10)]
    gs.append(synth.rmat_digraph(1 << 14, 1 << 18, synth.rng_for(61, 0), reciprocity=0.2))   # hub tasks
    gs.append(synth.Digraph(0, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty"))
    gs.append(synth.Digraph(3, np.array([0, 1, 2], np.int32), np.array([1, 2, 0], np.int32), "3-cycle"))
    return gs


def test_noalloc_equals_each_twice():
    pool = _pool()
    with tc.Context(0) as c:
        hs = [c.build_graph(g.n, g.src, g.dst) for g in pool]
        try:
            say(f"[gpu] noalloc: first call, {len(hs)} graphs")
            want = c.census_each(hs)
            got = c.census_each_noalloc(hs)
            assert got.tolist() == want.tolist()
            assert got[-1].tolist()[9] == 1                      # the 3-cycle is one 030C
            assert got[10].tolist() == oracle.census(pool[10].n, pool[10].src, pool[10].dst).tolist()
            # second call: fewer, smaller graphs; the array keeps the first call's
            # contents, so every block must be cleared again
            small = [hs[i] for i in (12, 2, 5)]
            say(f"[gpu] noalloc: second call, {len(small)} graphs")
            got2 = c.census_each_noalloc(small)
            assert got2.tolist() == c.census_each(small).tolist()
            for k, i in enumerate((12, 2, 5)):
                g = pool[i]
                assert got2[k].tolist() == oracle.census(g.n, g.src, g.dst).tolist(), g.name
            # through the dyad records as well
            default = c.get_tuning()
            c.set_tuning(**dict(default, tri=0))
            for h in hs:
                c.rebucket(h)
            say("[gpu] noalloc: dyad records")
            assert c.census_each_noalloc(hs).tolist() == want.tolist()
            c.set_tuning(**default)
            # limits: the most graphs one call takes, and one more
            say("[gpu] noalloc: size limit")
            many = [hs[k % 4] for k in range(tc.TC_NOALLOC_MAX_GRAPHS)]
            assert c.census_each_noalloc(many).tolist() == [want[k % 4].tolist() for k in range(len(many))]
            with pytest.raises(tc.TcError) as e:
                c.census_each_noalloc(many + [hs[0]])
            assert e.value.code == tc.TC_ERR_RANGE
            assert c.census_each_noalloc([]).shape == (0, 16)
        finally:
            for h in hs:
                h.release()
