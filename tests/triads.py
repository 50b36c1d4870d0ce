"""Test-side facts about 3-vertex digraphs, written from the class definitions
(MAN naming: M mutual, A asymmetric, N null dyads; letters D down, U up,
C cyclic, T transitive) and independent of both the oracle and the GPU library.

A triad is given by its 6-bit TriadCode: bit 1 u->v, 2 v->u, 4 u->w, 8 w->u,
16 v->w, 32 w->v, with u, v, w the vertices 0, 1, 2.
"""
from __future__ import annotations

import itertools
from math import comb

import numpy as np

NAMES = ("003", "012", "102", "021D", "021U", "021C", "111D", "111U",
         "030T", "030C", "201", "120D", "120U", "120C", "210", "300")
INDEX = {name: i for i, name in enumerate(NAMES)}

_ARC_BIT = {(0, 1): 1, (1, 0): 2, (0, 2): 4, (2, 0): 8, (1, 2): 16, (2, 1): 32}


def arcs_of(code: int):
    return [a for a, b in _ARC_BIT.items() if code & b]


def code_of(arcs) -> int:
    c = 0
    for a in arcs:
        c |= _ARC_BIT[a]
    return c


def permute(code: int, p) -> int:
    return code_of([(p[x], p[y]) for x, y in arcs_of(code)])


def transpose(code: int) -> int:
    return code_of([(y, x) for x, y in arcs_of(code)])


def complement(code: int) -> int:
    return 63 ^ code


def man(code: int):
    """(mutual, asymmetric, null) dyad counts."""
    a = set(arcs_of(code))
    m = s = 0
    for x, y in ((0, 1), (0, 2), (1, 2)):
        f, b = (x, y) in a, (y, x) in a
        if f and b:
            m += 1
        elif f or b:
            s += 1
    return m, s, 3 - m - s


def classify(code: int) -> int:
    """Class index by the naming rules (not by canonical forms)."""
    arcs = set(arcs_of(code))
    m, s, n = man(code)
    out = [sum(1 for (x, _) in arcs if x == v) for v in range(3)]
    inn = [sum(1 for (_, y) in arcs if y == v) for v in range(3)]
    base = f"{m}{s}{n}"
    if base in ("003", "012", "102", "201", "210", "300"):
        return INDEX[base]
    if base == "021":
        if 2 in out:
            return INDEX["021D"]
        if 2 in inn:
            return INDEX["021U"]
        return INDEX["021C"]
    if base == "111":
        pair = next(p for p in ((0, 1), (0, 2), (1, 2)) if p in arcs and p[::-1] in arcs)
        tail, head = next((x, y) for (x, y) in arcs if (y, x) not in arcs)
        return INDEX["111D"] if head in pair else INDEX["111U"]
    if base == "030":
        return INDEX["030C"] if out == [1, 1, 1] else INDEX["030T"]
    if base == "120":
        pair = next(p for p in ((0, 1), (0, 2), (1, 2)) if p in arcs and p[::-1] in arcs)
        r = 3 - pair[0] - pair[1]
        r_out = sum(1 for (x, y) in arcs if x == r)
        if r_out == 2:
            return INDEX["120D"]
        if r_out == 0:
            return INDEX["120U"]
        return INDEX["120C"]
    raise AssertionError(code)


RULE_TABLE = np.array([classify(c) for c in range(64)], dtype=np.uint8)


def brute_census(n: int, src, dst) -> np.ndarray:
    """Every triple classified by the rules above (pure Python; tiny n only)."""
    arcs = {(int(a), int(b)) for a, b in zip(src, dst) if a != b}
    out = np.zeros(16, np.uint64)
    for a, b, c in itertools.combinations(range(n), 3):
        code = 0
        for (x, y), bitv in _ARC_BIT.items():
            if ((a, b, c)[x], (a, b, c)[y]) in arcs:
                code |= bitv
        out[RULE_TABLE[code]] += 1
    return out


def counting_roles(a: int, b: int, c: int, joined) -> tuple | None:
    """Roles (u, v, w) in which the subquadratic loop counts the triple
    a < b < c with a third vertex, or None if no dyad of it is joined.

    Derived from the loop's condition (w counted for dyad (u, v), u < v, iff
    w in N(u) with w > v, or w in N(v) \\ N(u) with w > u): from dyad (a, b)
    the vertex c is counted iff c touches a or b; from (a, c) the vertex b is
    counted iff b touches c and not a; from (b, c) the vertex a never is.  A
    triple with one joined dyad is counted by that dyad's n - |S| - 2 term."""
    ab, ac, bc = joined(a, b), joined(a, c), joined(b, c)
    if ab:
        return (a, b, c)
    if ac:
        return (a, c, b)
    if bc:
        return (b, c, a)
    return None


def brute_census64(n: int, src, dst) -> np.ndarray:
    """64-class labelled census by triples (pure Python; tiny n only): the
    6-bit code of each triple read in the roles of counting_roles."""
    arcs = {(int(x), int(y)) for x, y in zip(src, dst) if x != y}

    def joined(x, y):
        return (x, y) in arcs or (y, x) in arcs

    out = np.zeros(64, np.uint64)
    for a, b, c in itertools.combinations(range(n), 3):
        roles = counting_roles(a, b, c, joined)
        code = 0
        if roles is not None:
            for (x, y), bitv in _ARC_BIT.items():
                if (roles[x], roles[y]) in arcs:
                    code |= bitv
        out[code] += 1
    return out


# ---- multiplicities for the exact degree identities ----------------------

def _per_class(fn):
    vals = [None] * 16
    for code in range(64):
        k = int(RULE_TABLE[code])
        v = fn(code)
        assert vals[k] is None or vals[k] == v, "not an isomorphism invariant"
        vals[k] = v
    return np.array(vals, dtype=object)


def _undirected_deg(code):
    a = set(arcs_of(code))
    return [sum(1 for w in range(3) if w != v and ((v, w) in a or (w, v) in a)) for v in range(3)]


MUL_M = _per_class(lambda c: man(c)[0])
MUL_A = _per_class(lambda c: man(c)[1])
MUL_N = _per_class(lambda c: man(c)[2])
MUL_WEDGE = _per_class(lambda c: sum(1 for d in _undirected_deg(c) if d == 2))
MUL_OUT2 = _per_class(lambda c: sum(1 for v in range(3) if sum(1 for (x, _) in arcs_of(c) if x == v) == 2))
MUL_IN2 = _per_class(lambda c: sum(1 for v in range(3) if sum(1 for (_, y) in arcs_of(c) if y == v) == 2))


def _paths2(c):
    a = set(arcs_of(c))
    tot = 0
    for v in range(3):
        ins = [x for (x, y) in a if y == v]
        outs = [y for (x, y) in a if x == v]
        tot += sum(1 for x in ins for y in outs if x != y)
    return tot


MUL_PATH2 = _per_class(_paths2)


def degree_sides(n: int, src, dst) -> dict:
    """Left-hand sides of the identities, computed from degrees in O(n + m)."""
    s = np.asarray(src, np.int64)
    d = np.asarray(dst, np.int64)
    keep = s != d
    k = np.unique(s[keep] * n + d[keep])
    s, d = k // n, k % n
    outd = np.bincount(s, minlength=n).astype(object)
    ind = np.bincount(d, minlength=n).astype(object)
    rk = d * n + s
    mutual_arc = np.isin(rk, k)
    mut = np.bincount(s[mutual_arc], minlength=n).astype(object)  # mutual partners of v
    und = outd + ind - mut
    M = int(mutual_arc.sum()) // 2
    A = int(k.size) - 2 * M
    pairs_total = n * (n - 1) // 2
    return dict(
        M=M, A=A, N=pairs_total - M - A,
        wedge=int(sum(comb(int(x), 2) for x in und)),
        out2=int(sum(comb(int(x), 2) for x in outd)),
        in2=int(sum(comb(int(x), 2) for x in ind)),
        path2=int(sum(int(i) * int(o) - int(m) for i, o, m in zip(ind, outd, mut))),
    )


def identity_violations(n: int, src, dst, census) -> list:
    """Returns the list of identities (I1..I5) the census violates."""
    c = np.array([int(x) for x in census], dtype=object)
    sides = degree_sides(n, src, dst)
    bad = []
    if int(c.sum()) != comb(n, 3):
        bad.append("I1 sum = C(n,3)")
    if int((MUL_M * c).sum()) != sides["M"] * (n - 2):
        bad.append("I2 mutual")
    if int((MUL_A * c).sum()) != sides["A"] * (n - 2):
        bad.append("I2 asymmetric")
    if int((MUL_N * c).sum()) != sides["N"] * (n - 2):
        bad.append("I2 null")
    if int((MUL_WEDGE * c).sum()) != sides["wedge"]:
        bad.append("I3 wedges")
    if int((MUL_OUT2 * c).sum()) != sides["out2"]:
        bad.append("I4 out-pairs")
    if int((MUL_IN2 * c).sum()) != sides["in2"]:
        bad.append("I4 in-pairs")
    if int((MUL_PATH2 * c).sum()) != sides["path2"]:
        bad.append("I5 two-paths")
    return bad
