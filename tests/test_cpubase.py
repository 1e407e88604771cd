"""The multithreaded CPU baseline the benchmark times computes the same
results as the oracle: BFS depths bit-exact, FP32 PageRank within L1 1e-5
after 20 iterations (FP32 row sums on the CPU)."""
import numpy as np
import pytest

import cpubase
import graphgen as gg
import oracle
from tests import graphs

CASES = [graphs.cycle(7), graphs.edgeless(5), graphs.star_in(9), graphs.chain(8), graphs.dangling_mix(),
         graphs.two_components(), graphs.random_small(64, 300, 1), gg.rmat(12, 16, seed=1), gg.grid(40, 50, 0.05, 3),
         gg.uniform(3000, 9000, seed=4)]


@pytest.mark.parametrize("g", CASES, ids=lambda g: g.name)
def test_bfs_matches_oracle(g):
    cg = cpubase.Graph(g.n, g.rowptr, g.colidx)
    for s in sorted({0, g.n - 1, g.n // 2}):
        got, secs = cg.bfs(s)
        np.testing.assert_array_equal(got, oracle.bfs(g.n, g.rowptr, g.colidx, s))
        assert secs >= 0.0


@pytest.mark.parametrize("g", CASES, ids=lambda g: g.name)
def test_pagerank_matches_oracle(g):
    cg = cpubase.Graph(g.n, g.rowptr, g.colidx)
    got, _ = cg.pagerank(20)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, r0=np.full(g.n, np.float32(1.0 / g.n), np.float64))
    assert float(np.abs(got.astype(np.float64) - want).sum()) <= 1e-5


def test_transpose_is_the_in_arc_csr():
    g = gg.rmat(10, 8, seed=2)
    cg = cpubase.Graph(g.n, g.rowptr, g.colidx)
    t_rowptr, t_colidx, _ = oracle.transpose(g.n, g.rowptr, g.colidx)
    np.testing.assert_array_equal(cg.t_rowptr, t_rowptr)
    np.testing.assert_array_equal(cg.t_colidx[:g.m], t_colidx)
