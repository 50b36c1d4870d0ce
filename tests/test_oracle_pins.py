"""Pins of the CPU oracle against facts the thesis and the mathematics fix.

None of these checks re-types the oracle's formulas: the table is checked
against group orbits, dyad counts read off the class names, and the
transpose/complement structure; the census is checked against the thesis's
worked graph, closed forms, a rule-based brute force written in Python, the
oracle's own O(n^3) count, exact degree identities, and symmetries.
"""
from math import comb
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_1603_02655_amd import synth
from tests import triads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build()


def C(**kw):
    out = np.zeros(16, np.uint64)
    for name, val in kw.items():
        out[triads.INDEX[name.lstrip("_")]] = val
    return out


def census(n, arcs):
    arcs = list(arcs)
    src = [a for a, _ in arcs]
    dst = [b for _, b in arcs]
    return oracle.census(n, src, dst)


# ---------------------------------------------------------------- table ----

def test_class_names_match_thesis_order():
    assert oracle.CLASS_NAMES == triads.NAMES


def test_table_class_sizes():
    t = oracle.table()
    sizes = np.bincount(t, minlength=16)
    assert sizes.tolist() == [1, 6, 3, 3, 3, 6, 6, 6, 6, 2, 3, 3, 3, 6, 6, 1]


def test_table_classes_are_relabelling_orbits():
    t = oracle.table()
    for code in range(64):
        orbit = {triads.permute(code, p) for p in itertools.permutations(range(3))}
        members = {c for c in range(64) if t[c] == t[code]}
        assert orbit == members, code


def test_table_dyad_counts_match_names():
    t = oracle.table()
    for code in range(64):
        name = triads.NAMES[t[code]]
        assert triads.man(code) == (int(name[0]), int(name[1]), int(name[2])), (code, name)


def test_table_matches_naming_rules():
    assert oracle.table().tolist() == triads.RULE_TABLE.tolist()


def test_table_transpose_swaps_down_and_up():
    t = oracle.table()
    swap = {"021D": "021U", "111D": "111U", "120D": "120U"}
    swap.update({v: k for k, v in swap.items()})
    for code in range(64):
        a = triads.NAMES[t[code]]
        b = triads.NAMES[t[triads.transpose(code)]]
        assert b == swap.get(a, a), (code, a, b)


def test_table_complement_map():
    t = oracle.table()
    comp = {"003": "300", "012": "210", "102": "201", "021D": "120U", "021U": "120D",
            "021C": "120C", "111D": "111D", "111U": "111U", "030T": "030T", "030C": "030C"}
    comp.update({v: k for k, v in comp.items()})
    for code in range(64):
        a = triads.NAMES[t[code]]
        b = triads.NAMES[t[triads.complement(code)]]
        assert b == comp[a], (code, a, b)


# ------------------------------------------------------- worked example ----

def load_golden():
    rows, counts = [], None
    with open(os.path.join(GOLDEN, "paper_adjmatrix.txt")) as f:
        lines = [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]
    i = lines.index("matrix") + 1
    while not lines[i].startswith("census"):
        rows.append([int(x) for x in lines[i].split()])
        i += 1
    names = lines[i].split()[1:]
    counts = [int(x) for x in lines[i + 1].split()]
    assert tuple(names) == triads.NAMES
    return np.array(rows), np.array(counts, np.uint64)


def test_paper_adjacency_matrix_example():
    mat, expected = load_golden()
    src, dst = np.nonzero(mat)
    assert mat[4, 4] == 1  # the example carries a loop; it is dropped
    got = oracle.census(mat.shape[0], src, dst)
    assert got.tolist() == expected.tolist()
    assert oracle.brute(mat.shape[0], src, dst).tolist() == expected.tolist()
    assert triads.brute_census(mat.shape[0], src, dst).tolist() == expected.tolist()


# ---------------------------------------------------------- closed forms ----

@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 17])
def test_empty_graph(n):
    assert census(n, []).tolist() == C(_003=comb(n, 3)).tolist()


@pytest.mark.parametrize("n", [3, 4, 9, 23])
def test_complete_digraph(n):
    arcs = [(a, b) for a in range(n) for b in range(n) if a != b]
    assert census(n, arcs).tolist() == C(_300=comb(n, 3)).tolist()


def test_three_cycle():
    assert census(3, [(0, 1), (1, 2), (2, 0)]).tolist() == C(_030C=1).tolist()


@pytest.mark.parametrize("n", [4, 5, 8, 31])
def test_directed_cycle(n):
    arcs = [(i, (i + 1) % n) for i in range(n)]
    exp = C(_021C=n, _012=n * (n - 4), _003=comb(n, 3) - n * (n - 3))
    assert census(n, arcs).tolist() == exp.tolist()


@pytest.mark.parametrize("n", [4, 6, 13])
def test_mutual_ring(n):
    arcs = [(i, (i + 1) % n) for i in range(n)] + [((i + 1) % n, i) for i in range(n)]
    exp = C(_201=n, _102=n * (n - 4), _003=comb(n, 3) - n * (n - 3))
    assert census(n, arcs).tolist() == exp.tolist()


@pytest.mark.parametrize("n", [3, 7, 20])
def test_transitive_tournament(n):
    arcs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    assert census(n, arcs).tolist() == C(_030T=comb(n, 3)).tolist()


@pytest.mark.parametrize("n", [3, 6, 40])
def test_stars(n):
    out_star = [(0, i) for i in range(1, n)]
    in_star = [(i, 0) for i in range(1, n)]
    assert census(n, out_star).tolist() == C(_021D=comb(n - 1, 2), _003=comb(n - 1, 3)).tolist()
    assert census(n, in_star).tolist() == C(_021U=comb(n - 1, 2), _003=comb(n - 1, 3)).tolist()


@pytest.mark.parametrize("n", [3, 10])
def test_single_arc_and_single_mutual(n):
    assert census(n, [(1, 2)]).tolist() == C(_012=n - 2, _003=comb(n, 3) - (n - 2)).tolist()
    assert census(n, [(1, 2), (2, 1)]).tolist() == C(_102=n - 2, _003=comb(n, 3) - (n - 2)).tolist()


@pytest.mark.parametrize("n", [3, 4, 5, 12])
def test_directed_and_mutual_path(n):
    # path 0 - 1 - ... - n-1: the n-2 consecutive triples hold two joined
    # pairs; arc (i, i+1) with a third vertex joined to neither: n-2 choices
    # less i-1 (when i >= 1) and i+2 (when i <= n-3), (n-2)(n-3) in all
    path = [(i, i + 1) for i in range(n - 1)]
    rest = comb(n, 3) - (n - 2) - (n - 2) * (n - 3)
    assert census(n, path).tolist() == C(_021C=n - 2, _012=(n - 2) * (n - 3), _003=rest).tolist()
    mutual = path + [(b, a) for a, b in path]
    assert census(n, mutual).tolist() == C(_201=n - 2, _102=(n - 2) * (n - 3), _003=rest).tolist()


@pytest.mark.parametrize("n", [3, 5, 30])
def test_mutual_star(n):
    arcs = [(0, i) for i in range(1, n)] + [(i, 0) for i in range(1, n)]
    assert census(n, arcs).tolist() == C(_201=comb(n - 1, 2), _003=comb(n - 1, 3)).tolist()


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (4, 2), (5, 7)])
def test_complete_bipartite(a, b):
    # every arc from side A (0..a-1) to side B: two A vertices with one of B
    # send both arcs to it (021U), one of A with two of B sends both (021D);
    # with every arc mutual both mixed kinds are two mutual pairs (201)
    A, B = range(a), range(a, a + b)
    one_way = [(x, y) for x in A for y in B]
    same_side = comb(a, 3) + comb(b, 3)
    assert census(a + b, one_way).tolist() == C(_021U=comb(a, 2) * b, _021D=a * comb(b, 2), _003=same_side).tolist()
    both = one_way + [(y, x) for x, y in one_way]
    assert census(a + b, both).tolist() == C(_201=comb(a, 2) * b + a * comb(b, 2), _003=same_side).tolist()


@pytest.mark.parametrize("a,b,c", [(1, 1, 1), (2, 1, 3), (3, 4, 2), (5, 2, 4)])
def test_layered_transitive_and_chain(a, b, c):
    # three layers A, B, C; every arc A->B and B->C, and for the transitive
    # form also A->C.  A triple is named by how many vertices it takes from
    # each layer.
    A, B, Cl = range(a), range(a, a + b), range(a + b, a + b + c)
    ab = [(x, y) for x in A for y in B]
    bc = [(y, z) for y in B for z in Cl]
    ac = [(x, z) for x in A for z in Cl]
    n = a + b + c
    same = comb(a, 3) + comb(b, 3) + comb(c, 3)
    # transitive: one per layer is 030T; two from an earlier layer and one
    # from a later one is 021U (both arcs into the later vertex), one from an
    # earlier layer and two from a later one is 021D
    exp = C(_030T=a * b * c,
            _021U=comb(a, 2) * (b + c) + comb(b, 2) * c,
            _021D=a * comb(b, 2) + a * comb(c, 2) + b * comb(c, 2),
            _003=same)
    assert census(n, ab + bc + ac).tolist() == exp.tolist()
    # chain (no A->C arcs): one per layer is the path A->B->C (021C); A and C
    # vertices alone are not joined (003)
    exp = C(_021C=a * b * c,
            _021U=comb(a, 2) * b + comb(b, 2) * c,
            _021D=a * comb(b, 2) + b * comb(c, 2),
            _003=same + comb(a, 2) * c + a * comb(c, 2))
    assert census(n, ab + bc).tolist() == exp.tolist()


@pytest.mark.parametrize("seed", range(4))
def test_random_tournament_kendall(seed):
    rng = np.random.default_rng(seed)
    n = 25
    arcs = []
    for a in range(n):
        for b in range(a + 1, n):
            arcs.append((a, b) if rng.random() < 0.5 else (b, a))
    score = np.bincount([a for a, _ in arcs], minlength=n)
    t = sum(comb(int(s), 2) for s in score)
    assert census(n, arcs).tolist() == C(_030T=t, _030C=comb(n, 3) - t).tolist()


# ----------------------------------------------------------- brute force ----

def _random_digraph(rng, n, p, mutual_boost):
    mat = rng.random((n, n)) < p
    recip = rng.random((n, n)) < mutual_boost
    mat |= mat.T & recip
    np.fill_diagonal(mat, rng.random(n) < 0.2)  # a few loops to be dropped
    src, dst = np.nonzero(mat)
    # duplicate some arcs: E is a set, duplicates must not count twice
    k = max(1, len(src) // 5)
    idx = rng.integers(0, max(1, len(src)), size=k) if len(src) else np.zeros(0, int)
    return np.concatenate([src, src[idx]]), np.concatenate([dst, dst[idx]])


@pytest.mark.parametrize("seed", range(40))
def test_oracle_vs_python_brute_tiny(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(0, 12))
    src, dst = _random_digraph(rng, n, rng.uniform(0, 1), rng.uniform(0, 1))
    want = triads.brute_census(n, src, dst)
    assert oracle.census(n, src, dst).tolist() == want.tolist()
    assert oracle.brute(n, src, dst).tolist() == want.tolist()


@pytest.mark.parametrize("seed", range(30))
def test_oracle_vs_brute_small(seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(3, 41))
    src, dst = _random_digraph(rng, n, rng.uniform(0, 0.6), rng.uniform(0, 1))
    want = oracle.brute(n, src, dst)
    got = oracle.census(n, src, dst)
    assert got.tolist() == want.tolist()
    assert triads.identity_violations(n, src, dst, got) == []


@pytest.mark.slow
def test_oracle_vs_brute_er_2000():
    g = synth.config_er_small()
    got = oracle.census(g.n, g.src, g.dst)
    want = oracle.brute(g.n, g.src, g.dst, threads=os.cpu_count() or 1)
    assert got.tolist() == want.tolist()
    assert triads.identity_violations(g.n, g.src, g.dst, got) == []


# ------------------------------------------------- identities, symmetries ----

def _rmat(n, m, seed, r=0.2, permute=True):
    return synth.rmat_digraph(n, m, synth.rng_for(90, seed), reciprocity=r, permute=permute)


@pytest.mark.parametrize("seed", range(3))
def test_degree_identities_rmat(seed):
    g = _rmat(3000, 30000, seed)
    got = oracle.census(g.n, g.src, g.dst)
    assert triads.identity_violations(g.n, g.src, g.dst, got) == []


def test_identities_catch_a_planted_error():
    g = _rmat(500, 4000, 7)
    got = oracle.census(g.n, g.src, g.dst).astype(object)
    for k in range(1, 16):
        bad = got.copy()
        bad[k] += 1
        bad[0] -= 1
        assert triads.identity_violations(g.n, g.src, g.dst, bad) != [], triads.NAMES[k]


def test_relabel_invariance():
    g = _rmat(2000, 16000, 3, permute=False)
    h = synth.relabel(g, np.random.default_rng(5))
    assert oracle.census(g.n, g.src, g.dst).tolist() == oracle.census(h.n, h.src, h.dst).tolist()


def test_transpose_swaps_d_and_u():
    g = _rmat(1500, 12000, 4)
    a = oracle.census(g.n, g.src, g.dst)
    b = oracle.census(g.n, g.dst, g.src)
    perm = list(range(16))
    for x, y in (("021D", "021U"), ("111D", "111U"), ("120D", "120U")):
        i, j = triads.INDEX[x], triads.INDEX[y]
        perm[i], perm[j] = j, i
    assert b.tolist() == a[perm].tolist()


def test_complement_on_small_graph():
    rng = np.random.default_rng(11)
    n = 30
    mat = rng.random((n, n)) < 0.3
    np.fill_diagonal(mat, False)
    src, dst = np.nonzero(mat)
    cs, cd = np.nonzero(~mat & ~np.eye(n, dtype=bool))
    a = oracle.census(n, src, dst)
    b = oracle.census(n, cs, cd)
    comp = {"003": "300", "012": "210", "102": "201", "021D": "120U", "021U": "120D",
            "021C": "120C", "111D": "111D", "111U": "111U", "030T": "030T", "030C": "030C"}
    comp.update({v: k for k, v in comp.items()})
    for name, k in triads.INDEX.items():
        assert int(b[triads.INDEX[comp[name]]]) == int(a[k])


def test_disjoint_union():
    g1 = _rmat(700, 5000, 21)
    g2 = _rmat(900, 7000, 22)
    c1 = oracle.census(g1.n, g1.src, g1.dst).astype(object)
    c2 = oracle.census(g2.n, g2.src, g2.dst).astype(object)
    n = g1.n + g2.n
    u = oracle.census(n, np.concatenate([g1.src, g2.src + g1.n]),
                      np.concatenate([g1.dst, g2.dst + g1.n])).astype(object)
    s1 = triads.degree_sides(g1.n, g1.src, g1.dst)
    s2 = triads.degree_sides(g2.n, g2.src, g2.dst)
    exp = c1 + c2
    exp[1] += s1["A"] * g2.n + s2["A"] * g1.n
    exp[2] += s1["M"] * g2.n + s2["M"] * g1.n
    exp[0] = comb(n, 3) - int(exp[1:].sum())
    assert u.tolist() == exp.tolist()


# ------------------------------------------------- task queues and threads ----

def test_range_census_sums_to_full():
    g = _rmat(4000, 40000, 9)
    with oracle.OracleGraph(g.n, g.src, g.dst) as og:
        full = og.census()
        cuts = [0, 17, 900, 901, 2500, g.n]
        parts = sum(og.census_range(a, b).astype(object) for a, b in zip(cuts, cuts[1:]))
        assert parts[0] == 0
        assert [int(x) for x in parts[1:]] == [int(x) for x in full[1:]]
        assert og.census_range(5, 5).tolist() == [0] * 16


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_multithreaded_equals_single(threads):
    g = _rmat(5000, 50000, 10)
    with oracle.OracleGraph(g.n, g.src, g.dst) as og:
        assert og.census_mt(threads).tolist() == og.census().tolist()


def test_bad_ids_rejected():
    with pytest.raises(ValueError):
        oracle.census(3, [0, 1], [1, 3])
    with pytest.raises(ValueError):
        oracle.census(3, [-1], [1])
