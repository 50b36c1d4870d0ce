"""The oracle's class labels against an independent, published implementation.

The thesis's figure of the 16 triad types is missing, so the names of the
three direction-sensitive pairs (021D/021U, 111D/111U, 120D/120U) rest on the
usual Batagelj-Mrvar convention, which the thesis inherits through its sources
(section "Triad Census Algorithm").  networkx's ``triadic_census`` implements
Batagelj and Mrvar's algorithm with their class names; the oracle must agree
with it on random digraphs and on single triads that tell each pair apart.
"""
import numpy as np
import pytest

import oracle
from tests import triads

nx = pytest.importorskip("networkx")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def _nx_census(n, src, dst):
    g = nx.DiGraph()
    g.add_nodes_from(range(n))
    g.add_edges_from((int(a), int(b)) for a, b in zip(src, dst) if a != b)
    c = nx.triadic_census(g)
    return [int(c[name]) for name in triads.NAMES]


# one triad per class on vertices a = 0, b = 1, c = 2, each written from its
# class's definition (x->y an arc, x<->y a mutual pair)
DISCRIMINATING = {
    "021D": [(1, 0), (1, 2)],                       # b->a, b->c: out-star
    "021U": [(0, 1), (2, 1)],                       # a->b, c->b: in-star
    "111D": [(0, 1), (1, 0), (2, 1)],               # a<->b, the arc c->b enters the pair
    "111U": [(0, 1), (1, 0), (1, 2)],               # a<->b, the arc b->c leaves the pair
    "120D": [(1, 0), (1, 2), (0, 2), (2, 0)],       # b->a, b->c, a<->c
    "120U": [(0, 1), (2, 1), (0, 2), (2, 0)],       # a->b, c->b, a<->c
}


@pytest.mark.parametrize("name", sorted(DISCRIMINATING))
def test_direction_sensitive_labels(name):
    arcs = DISCRIMINATING[name]
    src = [a for a, _ in arcs]
    dst = [b for _, b in arcs]
    want = [0] * 16
    want[triads.INDEX[name]] = 1
    assert _nx_census(3, src, dst) == want
    assert oracle.census(3, src, dst).tolist() == want
    # every relabelling of the three vertices keeps the label
    for perm in ([1, 2, 0], [2, 0, 1], [0, 2, 1]):
        ps = [perm[a] for a in src]
        pd = [perm[b] for b in dst]
        assert oracle.census(3, ps, pd).tolist() == want


def test_random_digraphs_agree_with_networkx():
    rng = np.random.default_rng(2013)
    for trial in range(200):
        n = int(rng.integers(3, 40))
        mat = rng.random((n, n)) < rng.uniform(0.02, 0.6)
        np.fill_diagonal(mat, False)
        src, dst = np.nonzero(mat)
        assert oracle.census(n, src, dst).tolist() == _nx_census(n, src, dst), trial


def test_sparse_rmat_agrees_with_networkx():
    from paper_1603_02655_amd import synth
    g = synth.rmat_digraph(3000, 12000, synth.rng_for(77, 0), reciprocity=0.2)
    assert oracle.census(g.n, g.src, g.dst).tolist() == _nx_census(g.n, g.src, g.dst)
