"""Randomized pins of the CPU oracle (no GPU): on random graphs, including
ones with isolated vertices, sinks and no arcs, each oracle function agrees
with an independent route to the same result: scipy's graph routines for
BFS, Dijkstra and the transpose, and the dense Google-matrix recurrence for
PageRank (uniform dangling mass) and the literal update without it."""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
from hypothesis import given, settings, strategies as st

import oracle

INT_MAX = np.iinfo(np.int32).max


def random_csr(n, m, seed, no_loops=True):
    """n vertices, up to m distinct arcs (duplicates merged), rows sorted."""
    rng = np.random.default_rng(seed)
    u = rng.integers(0, n, m).astype(np.int64)
    v = rng.integers(0, n, m).astype(np.int64)
    if no_loops:
        keep = u != v
        u, v = u[keep], v[keep]
    keys = np.unique(u * n + v)
    rows, cols = keys // n, (keys % n).astype(np.int32)
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=n))]).astype(np.int32)
    w = rng.integers(1, 256, cols.shape[0]).astype(np.int32)
    return rowptr, cols, w


def as_scipy(n, rowptr, cols, vals=None):
    data = np.ones(cols.shape[0]) if vals is None else vals.astype(np.float64)
    return sp.csr_matrix((data, cols, rowptr), shape=(n, n))


GRAPHS = dict(n=st.integers(1, 60), m=st.integers(0, 400), seed=st.integers(0, 2 ** 31))


@settings(max_examples=60, deadline=None, derandomize=True)
@given(**GRAPHS, src=st.integers(0, 10 ** 6))
def test_bfs_and_dijkstra_match_scipy(n, m, seed, src):
    rowptr, cols, w = random_csr(n, m, seed)
    s = src % n
    depth = oracle.bfs(n, rowptr, cols, s)
    want = csg.shortest_path(as_scipy(n, rowptr, cols), method="D", unweighted=True, indices=s)
    np.testing.assert_array_equal(depth, np.where(np.isinf(want), INT_MAX, want).astype(np.int64))
    dist = oracle.dijkstra(n, rowptr, cols, w, s)
    want = csg.dijkstra(as_scipy(n, rowptr, cols, w), indices=s)
    np.testing.assert_array_equal(dist, np.where(np.isinf(want), INT_MAX, want).astype(np.int64))


@settings(max_examples=60, deadline=None, derandomize=True)
@given(**GRAPHS)
def test_transpose_matches_scipy(n, m, seed):
    rowptr, cols, w = random_csr(n, m, seed)
    tr, tc, tw = oracle.transpose(n, rowptr, cols, w)
    want = as_scipy(n, rowptr, cols, w).T.tocsr()
    want.sort_indices()
    np.testing.assert_array_equal(tr, want.indptr)
    np.testing.assert_array_equal(tc, want.indices)
    np.testing.assert_array_equal(tw, want.data.astype(np.int32))


@settings(max_examples=40, deadline=None, derandomize=True)
@given(**GRAPHS, iters=st.integers(0, 12))
def test_pagerank_matches_dense_recurrence(n, m, seed, iters):
    rowptr, cols, _ = random_csr(n, m, seed)
    A = as_scipy(n, rowptr, cols).toarray()
    deg = A.sum(axis=1)
    M = np.zeros((n, n))
    nz = deg > 0
    M[:, nz] = (A[nz, :] / deg[nz, None]).T  # M[v, u] = 1 / outdeg(u) for u -> v
    r0 = np.random.default_rng(seed + 1).random(n)
    r0 /= r0.sum()
    d = 0.85
    # uniform: a dangling vertex's rank is spread over all vertices
    G = d * (M + np.outer(np.ones(n), ~nz) / n) + (1 - d) / n
    want = r0.copy()
    for _ in range(iters):
        want = G @ want
    got = oracle.pagerank(n, rowptr, cols, d, iters, mode=oracle.UNIFORM, r0=r0)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
    # leak: the literal update, dangling rank dropped
    want = r0.copy()
    for _ in range(iters):
        want = (1 - d) / n + d * (M @ want)
    got = oracle.pagerank(n, rowptr, cols, d, iters, mode=oracle.LEAK, r0=r0)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


@settings(max_examples=30, deadline=None, derandomize=True)
@given(n=st.integers(1, 30), m=st.integers(0, 150), seed=st.integers(0, 2 ** 31), n_src=st.integers(1, 6))
def test_bc_matches_networkx_subset(n, m, seed, n_src):
    import networkx as nx
    rowptr, cols, _ = random_csr(n, m, seed)
    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    src = np.repeat(np.arange(n), np.diff(rowptr))
    G.add_edges_from(zip(src.tolist(), cols.tolist()))
    sources = sorted(set(np.random.default_rng(seed + 7).integers(0, n, n_src).tolist()))
    want = nx.betweenness_centrality_subset(G, sources, list(range(n)), normalized=False)
    got = oracle.bc(n, rowptr, cols, sources)
    np.testing.assert_allclose(got, [want[v] for v in range(n)], rtol=1e-12, atol=1e-12)


@settings(max_examples=40, deadline=None, derandomize=True)
@given(**GRAPHS, iters=st.integers(0, 12))
def test_ppr_and_spmv_match_dense(n, m, seed, iters):
    rowptr, cols, _ = random_csr(n, m, seed)
    A = as_scipy(n, rowptr, cols).toarray()
    deg = A.sum(axis=1)
    M = np.zeros((n, n))
    nz = deg > 0
    M[:, nz] = (A[nz, :] / deg[nz, None]).T
    rng = np.random.default_rng(seed + 3)
    p = rng.random(n)
    p /= p.sum()
    d = 0.85
    # personalised: the teleport and the dangling mass both go to p
    want = p.copy()
    for _ in range(iters):
        want = (1 - d) * p + d * (M @ want + want[~nz].sum() * p)
    np.testing.assert_allclose(oracle.ppr(n, rowptr, cols, p, d, iters), want, rtol=0, atol=1e-13)
    vals = rng.uniform(-1.0, 1.0, cols.shape[0])
    x = rng.uniform(-1.0, 1.0, n)
    np.testing.assert_allclose(oracle.spmv(n, rowptr, cols, vals, x), as_scipy(n, rowptr, cols, vals).T @ x,
                               rtol=0, atol=1e-12)
