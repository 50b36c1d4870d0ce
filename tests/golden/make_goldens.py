"""Writes (and reads) the full-size census goldens: the oracle's 16-class
census of every full-size workload graph, stored once so that the GPU tests
can compare the whole 16-vector element by element at sizes the oracle takes
minutes on.

TEST INFRASTRUCTURE.  This script calls only the CPU oracle (``oracle/``) and
the seeded generators (``paper_1603_02655_amd/synth.py``, which hold no census
arithmetic); no stored value comes from the GPU library.

Files written under ``tests/golden/`` (one line per graph:
``name n arcs_in arc_hash c_003 ... c_300``, classes in the thesis's order,
section "Triad Census Algorithm"):

* ``census_rmat_2p20.txt``   R-MAT (0.57, 0.19, 0.19, 0.05), n = 2^20, 2^24
                             arcs, reciprocity 0.20 (multithreaded oracle);
* ``census_citation.txt``    the citation-shaped DAG, n = 3.8 M, 16.5 M arcs;
* ``census_batch_pool.txt``  all 4096 graphs of the batch pool (R-MAT, n
                             log-uniform in [50, 20000], mean out-degree
                             U[3, 30], reciprocity 0.10);
* ``census_serving_pool.txt`` the first 64 graphs of the serving pool (even
                             ER, odd R-MAT r = 0.10, n log-uniform [1e3, 1e6],
                             mean out-degree U[4, 32]).

``arc_hash`` is the first 16 hex digits of the SHA-256 of the tail array
followed by the head array (int32, little endian), as generated: a test
regenerates the graph and compares the hash before it compares counts, so a
change of the generators cannot pass as a census mismatch or a match.

    python tests/golden/make_goldens.py [rmat citation batch serve] [--threads T]
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FILES = {
    "rmat": "census_rmat_2p20.txt",
    "citation": "census_citation.txt",
    "batch": "census_batch_pool.txt",
    "serve": "census_serving_pool.txt",
}
BATCH_COUNT = 4096
SERVE_COUNT = 64

HEADERS = {
    "rmat": "R-MAT (0.57, 0.19, 0.19, 0.05), n = 2^20, 2^24 arcs, reciprocity 0.20, "
            "relabelled (synth.config_rmat_2p20)",
    "citation": "citation-shaped DAG, n = 3.8 M, 16.5 M arcs, reciprocity 0.5 % (synth.config_citation)",
    "batch": f"batch pool, graphs 0..{BATCH_COUNT - 1} (synth.batch_graph)",
    "serve": f"serving pool, graphs 0..{SERVE_COUNT - 1} (synth.serving_graph)",
}


def arc_hash(src, dst) -> str:
    """First 16 hex digits of SHA-256 over the int32 tails then heads."""
    import numpy as np
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(src, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(dst, dtype="<i4").tobytes())
    return h.hexdigest()[:16]


def load(kind: str) -> list:
    """Records of one golden file: dicts with name, n, m, hash, counts (16 ints)."""
    out = []
    with open(os.path.join(HERE, FILES[kind])) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            cells = line.split()
            out.append({"name": cells[0], "n": int(cells[1]), "m": int(cells[2]), "hash": cells[3],
                        "counts": [int(x) for x in cells[4:20]]})
    return out


def _graph(kind: str, i: int):
    from paper_1603_02655_amd import synth
    if kind == "rmat":
        return synth.config_rmat_2p20()
    if kind == "citation":
        return synth.config_citation()
    if kind == "batch":
        return synth.batch_graph(i)
    return synth.serving_graph(i)


def graph_with_hash(args):
    """(graph, arc hash) of graph i of one kind; args = (kind, i).  Top level so
    that worker processes can run it."""
    kind, i = args
    g = _graph(kind, i)
    return g, arc_hash(g.src, g.dst)


def _record(kind: str, i: int, threads: int) -> str:
    import oracle
    g = _graph(kind, i)
    with oracle.OracleGraph(g.n, g.src, g.dst) as og:
        c = og.census_mt(threads) if threads > 1 else og.census()
    name = g.name if kind in ("rmat", "citation") else f"{kind}-{i}"
    return " ".join([name, str(g.n), str(g.m), arc_hash(g.src, g.dst)] + [str(int(x)) for x in c])


def _pool_record(args):
    return _record(*args)


def write(kind: str, threads: int) -> None:
    t = time.perf_counter()
    if kind in ("rmat", "citation"):
        lines = [_record(kind, 0, threads)]
    else:
        count = BATCH_COUNT if kind == "batch" else SERVE_COUNT
        jobs = [(kind, i, 1) for i in range(count)]
        with ProcessPoolExecutor(max_workers=threads) as ex:
            lines = list(ex.map(_pool_record, jobs, chunksize=1 if kind == "serve" else 16))
    path = os.path.join(HERE, FILES[kind])
    with open(path + ".tmp", "w") as f:
        f.write(f"# Oracle census (oracle/oracle.c) of the {HEADERS[kind]}.\n")
        f.write("# Written by tests/golden/make_goldens.py, which calls only the CPU oracle and the\n")
        f.write("# seeded generators.  Columns: name n arcs_in arc_hash, then the 16 class counts\n")
        f.write("# 003 012 102 021D 021U 021C 111D 111U 030T 030C 201 120D 120U 120C 210 300\n")
        f.write("# (section \"Triad Census Algorithm\"; each row sums to C(n, 3)).\n")
        for ln in lines:
            f.write(ln + "\n")
    os.replace(path + ".tmp", path)
    print(f"{kind}: {len(lines)} graphs in {time.perf_counter() - t:.1f} s -> {path}", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("kinds", nargs="*", default=list(FILES))
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for k in a.kinds:
        write(k, a.threads)


if __name__ == "__main__":
    main()
