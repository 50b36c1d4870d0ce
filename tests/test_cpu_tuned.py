"""The multicore CPU census (libtc_cpu.so, a context baseline) against the
oracle: bit-exact counts on the thesis's worked graph, random tiny graphs
(also against the Python brute force), R-MAT and citation-shaped graphs, with
one and several threads."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1603_02655_amd import build as pkg_build
from paper_1603_02655_amd import cpu_census, synth
from tests import triads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(cpu_census.LIB_PATH):
        pkg_build.build_cpu()
    oracle.build() if not os.path.exists(oracle.LIB_PATH) else None


def test_exports_declared_symbols():
    text = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "tc_cpu.h")).read(), flags=re.S)
    names = set(re.findall(r"\b(tc_cpu_[a-z_0-9]+)\s*\(", text))
    lib = ctypes.CDLL(cpu_census.LIB_PATH)
    assert names and all(hasattr(lib, n) for n in names)


def test_paper_example():
    arcs = [(0, 1), (0, 2), (0, 3), (3, 4), (3, 5), (5, 3), (4, 4)]
    src, dst = [a for a, _ in arcs], [b for _, b in arcs]
    got, _ = cpu_census.census(7, src, dst, threads=2)
    assert got.tolist() == oracle.census(7, src, dst).tolist()


def test_tiny_random_vs_brute():
    rng = np.random.default_rng(11)
    for _ in range(25):
        n = int(rng.integers(3, 12))
        m = int(rng.integers(0, 3 * n))
        src, dst = rng.integers(0, n, m), rng.integers(0, n, m)
        got, _ = cpu_census.census(n, src, dst, threads=3)
        assert got.tolist() == triads.brute_census(n, src, dst).tolist()


@pytest.mark.parametrize("threads", [1, 4])
def test_rmat_and_citation_vs_oracle(threads):
    for g in (synth.rmat_digraph(1 << 12, 1 << 16, synth.rng_for(81, 0), reciprocity=0.2),
              synth.citation_dag(30000, 130000, synth.rng_for(81, 1))):
        got, secs = cpu_census.census(g.n, g.src, g.dst, threads=threads)
        assert secs >= 0.0
        assert got.tolist() == oracle.census(g.n, g.src, g.dst).tolist(), g.name


def test_errors_and_small_n():
    with pytest.raises(ValueError):
        cpu_census.census(3, [0, 1], [1, 5])
    for n in (0, 1, 2):
        got, _ = cpu_census.census(n, [], [])
        assert int(got.sum()) == 0
