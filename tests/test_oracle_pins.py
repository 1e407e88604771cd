"""Pins the CPU oracle to facts outside itself (no GPU).

Each check is a different route to the same number: dense linear algebra
(matrix powers, eigenvectors, linear solves), networkx / scipy library
routines, closed forms for special graphs, brute force on tiny graphs and
optimality certificates. A dropped term, a swapped index or a transposed
operand in the oracle fails at least one of them.
"""
import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen as gg
import oracle
from tests import graphs

D = 0.85


def dense_adj(g):
    """A[u, v] = 1 for every arc u -> v, built from the CSR arrays."""
    A = sp.csr_matrix((np.ones(g.m), g.colidx, g.rowptr), shape=(g.n, g.n)).toarray()
    return A


def google_matrix(g, d=D, mode=oracle.UNIFORM):
    """Column-stochastic (UNIFORM) operator r' = G r of the PageRank iteration."""
    A = dense_adj(g)
    n = g.n
    deg = A.sum(axis=1)
    M = np.zeros((n, n))
    nz = deg > 0
    M[:, nz] = (A[nz, :] / deg[nz, None]).T  # M[v, u] = 1/deg(u) for u -> v
    if mode == oracle.UNIFORM:
        M[:, ~nz] = 1.0 / n
    return d * M + (1.0 - d) / n * np.ones((n, n)), M


@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
def test_pagerank_20_steps_equals_dense_matrix_power(g):
    G, _ = google_matrix(g)
    r0 = np.full(g.n, 1.0 / g.n)
    want = np.linalg.matrix_power(G, 20) @ r0
    got = oracle.pagerank(g.n, g.rowptr, g.colidx, D, 20)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
def test_pagerank_leak_20_steps_equals_dense_recurrence(g):
    _, M = google_matrix(g, mode=oracle.LEAK)
    n = g.n
    r = np.full(n, 1.0 / n)
    for _ in range(20):
        r = D * M @ r + (1.0 - D) / n
    got = oracle.pagerank(n, g.rowptr, g.colidx, D, 20, mode=oracle.LEAK)
    np.testing.assert_allclose(got, r, rtol=0, atol=1e-13)


@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
def test_pagerank_fixed_point_is_principal_eigenvector(g):
    G, _ = google_matrix(g)
    w, V = np.linalg.eig(G)
    i = np.argmax(w.real)
    assert abs(w[i] - 1.0) < 1e-10
    v = np.abs(V[:, i].real)
    v /= v.sum()
    got = oracle.pagerank(g.n, g.rowptr, g.colidx, D, 400)
    np.testing.assert_allclose(got, v, rtol=0, atol=1e-12)


@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
def test_pagerank_fixed_point_solves_linear_system(g):
    A = dense_adj(g)
    n = g.n
    deg = A.sum(axis=1)
    M = np.zeros((n, n))
    nz = deg > 0
    M[:, nz] = (A[nz, :] / deg[nz, None]).T
    a = (~nz).astype(float)
    lhs = np.eye(n) - D * M - (D / n) * np.outer(np.ones(n), a)
    want = np.linalg.solve(lhs, np.full(n, (1.0 - D) / n))
    got = oracle.pagerank(n, g.rowptr, g.colidx, D, 400)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    # LEAK limit: (I - dM) r = (1-d)/n
    want_leak = np.linalg.solve(np.eye(n) - D * M, np.full(n, (1.0 - D) / n))
    got_leak = oracle.pagerank(n, g.rowptr, g.colidx, D, 400, mode=oracle.LEAK)
    np.testing.assert_allclose(got_leak, want_leak, rtol=0, atol=1e-12)


@pytest.mark.parametrize("g", [graphs.random_small(60, 240, 7), graphs.dangling_mix(),
                               gg.rmat(8, 8, seed=9)], ids=lambda g: g.name)
def test_pagerank_matches_networkx(g):
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    for u in range(g.n):
        for v in g.colidx[g.rowptr[u]:g.rowptr[u + 1]]:
            G.add_edge(u, int(v))
    ref = nx.pagerank(G, alpha=D, tol=1e-15, max_iter=100000)
    ref = np.array([ref[i] for i in range(g.n)])
    got = oracle.pagerank(g.n, g.rowptr, g.colidx, D, 400)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-11)


@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
def test_pagerank_sums_to_one_every_iteration(g):
    for t in range(1, 21):
        r = oracle.pagerank(g.n, g.rowptr, g.colidx, D, t)
        assert abs(r.sum() - 1.0) < 1e-12


def test_pagerank_closed_forms():
    for g in (graphs.cycle(11), graphs.complete(7), graphs.edgeless(9)):
        for t in (1, 5, 20):
            r = oracle.pagerank(g.n, g.rowptr, g.colidx, D, t)
            np.testing.assert_allclose(r, np.full(g.n, 1.0 / g.n), rtol=0, atol=1e-15)
    # LEAK on an edgeless graph: every step gives exactly (1-d)/n
    g = graphs.edgeless(5)
    r = oracle.pagerank(g.n, g.rowptr, g.colidx, D, 3, mode=oracle.LEAK)
    np.testing.assert_allclose(r, np.full(5, (1 - D) / 5), rtol=0, atol=1e-16)
    # star with hub in-arcs: hub = (1-d)/n + d*(sum of leaves) + dangling share
    g = graphs.star_in(5)
    r = oracle.pagerank(g.n, g.rowptr, g.colidx, D, 1)
    leaves = (1 - D) / 5 + D * (0.2 / 5)  # only the hub (dangling) spreads
    hub = (1 - D) / 5 + D * (4 * 0.2 + 0.2 / 5)
    np.testing.assert_allclose(r, [hub] + [leaves] * 4, rtol=0, atol=1e-16)


@pytest.mark.parametrize("g", [graphs.random_small(30, 90, 3), graphs.dangling_mix(),
                               gg.rmat(6, 8, seed=5)], ids=lambda g: g.name)
def test_ppr_fixed_point_solves_linear_system(g):
    n = g.n
    A = dense_adj(g)
    deg = A.sum(axis=1)
    M = np.zeros((n, n))
    nz = deg > 0
    M[:, nz] = (A[nz, :] / deg[nz, None]).T
    seed = int(np.argmax(deg))
    p = np.zeros(n)
    p[seed] = 1.0
    Mp = M.copy()
    Mp[:, ~nz] = p[:, None]  # dangling mass goes to p
    want = (1 - D) * np.linalg.solve(np.eye(n) - D * Mp, p)
    got = oracle.ppr(n, g.rowptr, g.colidx, p, D, 500)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)
    assert abs(got.sum() - 1.0) < 1e-12
    # 20-step iterate as a dense matrix power from r0 = p
    G = D * Mp + (1 - D) * np.outer(p, np.ones(n))
    np.testing.assert_allclose(oracle.ppr(n, g.rowptr, g.colidx, p, D, 20),
                               np.linalg.matrix_power(G, 20) @ p, rtol=0, atol=1e-13)


def _scipy_graph(g, weights=None):
    data = np.ones(g.m) if weights is None else weights.astype(np.float64)
    return sp.csr_matrix((data, g.colidx, g.rowptr), shape=(g.n, g.n))


def _as_int(d):
    out = np.full(d.shape, oracle.INF32, dtype=np.int64)
    fin = np.isfinite(d)
    out[fin] = d[fin].astype(np.int64)
    return out


@pytest.mark.parametrize("g", graphs.all_small() + [gg.rmat(12, 8, seed=1), gg.grid(40, 50, 0.05, seed=3),
                                                     gg.uniform(3000, 6000, seed=4)],
                         ids=lambda g: g.name)
def test_bfs_matches_scipy_and_networkx(g):
    srcs = sorted(set([0, g.n - 1] + list(gg.sources(g, 3, seed=11))))
    for s in srcs:
        got = oracle.bfs(g.n, g.rowptr, g.colidx, s)
        ref = csg.shortest_path(_scipy_graph(g), method="D", unweighted=True, indices=s)
        np.testing.assert_array_equal(got, _as_int(ref))
    if g.n <= 5000:
        G = nx.DiGraph()
        G.add_nodes_from(range(g.n))
        G.add_edges_from((u, int(v)) for u in range(g.n) for v in g.colidx[g.rowptr[u]:g.rowptr[u + 1]])
        lengths = nx.single_source_shortest_path_length(G, srcs[0])
        want = np.full(g.n, oracle.INF32, dtype=np.int64)
        for v, l in lengths.items():
            want[v] = l
        np.testing.assert_array_equal(oracle.bfs(g.n, g.rowptr, g.colidx, srcs[0]), want)


def floyd_warshall(g, weights):
    n = g.n
    INF = np.iinfo(np.int64).max // 4
    Dm = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(Dm, 0)
    for u in range(n):
        for j in range(g.rowptr[u], g.rowptr[u + 1]):
            v = g.colidx[j]
            Dm[u, v] = min(Dm[u, v], weights[j])
    for k in range(n):
        Dm = np.minimum(Dm, Dm[:, k:k + 1] + Dm[k:k + 1, :])
    Dm[Dm >= INF] = oracle.INF32
    return Dm


@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
def test_bfs_and_dijkstra_match_floyd_warshall(g):
    w = g.with_weights(17).weights
    Dw = floyd_warshall(g, w)
    Du = floyd_warshall(g, np.ones(g.m, dtype=np.int64))
    for s in range(g.n):
        np.testing.assert_array_equal(oracle.dijkstra(g.n, g.rowptr, g.colidx, w, s), Dw[s])
        np.testing.assert_array_equal(oracle.bfs(g.n, g.rowptr, g.colidx, s), Du[s])
        # BFS is Dijkstra with unit weights
        np.testing.assert_array_equal(oracle.bfs(g.n, g.rowptr, g.colidx, s),
                                      oracle.dijkstra(g.n, g.rowptr, g.colidx, np.ones(g.m, np.int32), s))


def sssp_certificate(g, w, s, dist):
    """Optimality certificate for positive weights (implementation free)."""
    INF = oracle.INF32
    assert dist[s] == 0
    src = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    dv, du = dist[g.colidx].astype(np.int64), dist[src].astype(np.int64)
    fin = du != INF
    assert np.all(dv[fin] <= du[fin] + w[fin])  # no arc can improve
    tight = fin & (dv == du + w)
    has_tight = np.zeros(g.n, bool)
    has_tight[g.colidx[tight]] = True
    reached = dist != INF
    reached[s] = False
    assert np.all(has_tight[reached])  # every reached v != s has a tight in-arc
    assert np.all(dist[g.colidx[fin]] != INF)  # nothing reachable left unreached


@pytest.mark.parametrize("g", [gg.rmat(12, 8, seed=1), gg.grid(64, 64, 0.05, seed=3),
                               gg.uniform(5000, 10000, seed=4), gg.rmat(10, 16, seed=2, permute=False)],
                         ids=lambda g: g.name)
def test_dijkstra_matches_scipy_and_certificate(g):
    w = g.with_weights(5).weights
    for s in gg.sources(g, 3, seed=13):
        got = oracle.dijkstra(g.n, g.rowptr, g.colidx, w, s)
        ref = csg.dijkstra(_scipy_graph(g, w), indices=s)
        np.testing.assert_array_equal(got, _as_int(ref))
        sssp_certificate(g, w, s, got)
        got_b = oracle.bfs(g.n, g.rowptr, g.colidx, s)
        sssp_certificate(g, np.ones(g.m, np.int64), s, got_b)


def test_dijkstra_rejects_nonpositive_weight():
    g = graphs.cycle(4)
    with pytest.raises(ValueError):
        oracle.dijkstra(g.n, g.rowptr, g.colidx, np.array([1, 0, 1, 1], np.int32), 0)


@pytest.mark.parametrize("g", graphs.all_small() + [gg.rmat(10, 8, seed=1)], ids=lambda g: g.name)
def test_transpose_matches_scipy(g):
    w = g.with_weights(3).weights
    tr, tc, tw = oracle.transpose(g.n, g.rowptr, g.colidx, w)
    T = _scipy_graph(g, w).T.tocsr()
    T.sort_indices()
    np.testing.assert_array_equal(tr, T.indptr)
    np.testing.assert_array_equal(tc, T.indices)
    np.testing.assert_array_equal(tw, T.data.astype(np.int32))


# ---- convergence-driven PageRank (the stopping rule of Section 4, read as an
# L1 test on the change between consecutive iterates) ----

@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
def test_converge_changes_shrink_by_the_damping(g):
    """With UNIFORM dangling the iteration map is r -> G r, G column-stochastic
    scaled by d plus a constant, so consecutive differences obey
    ||G x||_1 <= d ||x||_1: each delta is at most d times the one before."""
    _, k, deltas = oracle.pagerank_converge(g.n, g.rowptr, g.colidx, 0.0, 30, D)
    assert k == 30 or deltas[-1] == 0.0
    for a, b in zip(deltas, deltas[1:]):
        assert b <= D * a + 1e-15


@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
def test_converge_stops_at_first_small_change_within_the_contraction_bound(g):
    """Stops at the first k with delta_k <= tol, and the contraction bound
    ||r_k - r*||_1 <= d/(1-d) delta_k holds against the dense linear solve."""
    G, _ = google_matrix(g)
    n = g.n
    want = np.linalg.solve(np.eye(n) - (G - (1.0 - D) / n * np.ones((n, n))), np.full(n, (1.0 - D) / n))
    tol = 1e-7
    r, k, deltas = oracle.pagerank_converge(n, g.rowptr, g.colidx, tol, 1000, D)
    assert deltas[-1] <= tol and all(x > tol for x in deltas[:-1])
    assert np.abs(r - want).sum() <= D / (1.0 - D) * deltas[-1] + 1e-12
    # the iterate itself is the plain fixed-count one
    np.testing.assert_allclose(r, oracle.pagerank(n, g.rowptr, g.colidx, D, k), rtol=0, atol=1e-15)


def test_converge_closed_forms_and_cap():
    # a directed cycle keeps the uniform vector: the first change is exactly 0
    n = 12
    rowptr = np.arange(n + 1, dtype=np.int32)
    colidx = ((np.arange(n) + 1) % n).astype(np.int32)
    r, k, deltas = oracle.pagerank_converge(n, rowptr, colidx, 0.0, 50, D)
    assert (k, deltas) == (1, [0.0])
    np.testing.assert_allclose(r, np.full(n, 1.0 / n), rtol=0, atol=1e-16)
    # a star (all arcs into vertex 0, which has none) needs many steps; the cap holds
    rowptr = np.concatenate([[0, 0], np.arange(1, n, dtype=np.int32)]).astype(np.int32)
    colidx = np.zeros(n - 1, dtype=np.int32)
    _, k, deltas = oracle.pagerank_converge(n, rowptr, colidx, 0.0, 7, D)
    assert k == 7 and len(deltas) == 7 and deltas[-1] > 0.0


# ---- SpMV over the arcs in the pull direction (Section 4's SpMV benchmark) ----

@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
def test_spmv_matches_scipy_and_dense(g):
    rng = np.random.default_rng(5)
    vals = rng.uniform(-1.0, 1.0, g.m)
    x = rng.uniform(-1.0, 1.0, g.n)
    A = sp.csr_matrix((vals, g.colidx, g.rowptr), shape=(g.n, g.n))
    got = oracle.spmv(g.n, g.rowptr, g.colidx, vals, x)
    np.testing.assert_allclose(got, A.T @ x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(got, A.toarray().T @ x, rtol=0, atol=1e-12)
    # unit values: the pull neighbour sum
    ones = oracle.spmv(g.n, g.rowptr, g.colidx, None, x)
    np.testing.assert_allclose(ones, (dense_adj(g).T @ x), rtol=0, atol=1e-12)


def test_spmv_linearity_and_pagerank_step():
    g = gg.rmat(9, 8, seed=4)
    rng = np.random.default_rng(6)
    vals = rng.uniform(0.0, 2.0, g.m)
    x, z = rng.uniform(-1, 1, g.n), rng.uniform(-1, 1, g.n)
    lhs = oracle.spmv(g.n, g.rowptr, g.colidx, vals, 2.0 * x - 3.0 * z)
    rhs = 2.0 * oracle.spmv(g.n, g.rowptr, g.colidx, vals, x) - 3.0 * oracle.spmv(g.n, g.rowptr, g.colidx, vals, z)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12)
    # with values 1 / outdeg(u) and x = r, one product is the neighbour sum of
    # a PageRank step: r' = (1-d)/n + d (s + D/n) (leak mode: no D term)
    deg = np.diff(g.rowptr)
    r = np.full(g.n, 1.0 / g.n)
    s = oracle.spmv(g.n, g.rowptr, g.colidx, np.repeat(1.0 / np.maximum(deg, 1), deg), r)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, D, 1, mode=oracle.LEAK)
    np.testing.assert_allclose((1.0 - D) / g.n + D * s, want, rtol=0, atol=1e-15)


# ---- betweenness centrality (Section 4's BC benchmark, Brandes' dependencies) ----

def _all_shortest_paths_bc(n, rowptr, colidx):
    """BC by explicit enumeration of every shortest path (tiny graphs only):
    for each (s, t) all simple s -> t paths are listed by depth-first search
    and the shortest kept; v scores the fraction of them passing through it."""
    adj = [list(colidx[rowptr[u]:rowptr[u + 1]]) for u in range(n)]
    out = np.zeros(n)
    for s in range(n):
        paths = {t: [] for t in range(n)}
        stack = [(s, [s])]
        while stack:
            u, p = stack.pop()
            paths[u].append(p)
            for v in adj[u]:
                if v not in p:
                    stack.append((v, p + [v]))
        for t in range(n):
            if t == s or not paths[t]:
                continue
            L = min(len(p) for p in paths[t])
            short = [p for p in paths[t] if len(p) == L]
            for p in short:
                for v in p[1:-1]:
                    out[v] += 1.0 / len(short)
    return out


@pytest.mark.parametrize("g", [graphs.random_small(9, 20, 3), graphs.random_small(8, 16, 11), graphs.dangling_mix(),
                               graphs.two_components(), graphs.cycle(7)], ids=lambda g: g.name)
def test_bc_matches_path_enumeration(g):
    if g.n > 10:
        pytest.skip("enumeration is for tiny graphs")
    got = oracle.bc(g.n, g.rowptr, g.colidx, range(g.n))
    np.testing.assert_allclose(got, _all_shortest_paths_bc(g.n, g.rowptr, g.colidx), rtol=0, atol=1e-12)


@pytest.mark.parametrize("g", [graphs.random_small(60, 240, 7), graphs.dangling_mix(), gg.rmat(8, 8, seed=9),
                               graphs.two_components()], ids=lambda g: g.name)
def test_bc_matches_networkx(g):
    G = nx.DiGraph()
    G.add_nodes_from(range(g.n))
    src = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    G.add_edges_from(zip(src.tolist(), g.colidx.tolist()))
    want = nx.betweenness_centrality(G, normalized=False)
    got = oracle.bc(g.n, g.rowptr, g.colidx, range(g.n))
    np.testing.assert_allclose(got, [want[v] for v in range(g.n)], rtol=1e-12, atol=1e-12)


def test_bc_closed_forms():
    # directed chain 0 -> 1 -> ... -> n-1: v lies on the one path of every
    # pair s < v < t, so BC(v) = v (n - 1 - v)
    n = 9
    rowptr = np.concatenate([np.arange(n), [n - 1]]).astype(np.int32)
    colidx = np.arange(1, n, dtype=np.int32)
    np.testing.assert_allclose(oracle.bc(n, rowptr, colidx, range(n)), [v * (n - 1 - v) for v in range(n)])
    # sigma on a 4 x 4 directed grid (right / down arcs) from the corner is
    # the binomial count of monotone lattice paths
    k = 4
    rows, cols = [], []
    for r in range(k):
        for c in range(k):
            u = r * k + c
            nb = ([u + 1] if c + 1 < k else []) + ([u + k] if r + 1 < k else [])
            rows.append(len(nb))
            cols += nb
    rowptr = np.concatenate([[0], np.cumsum(rows)]).astype(np.int32)
    _, sigma, depth = oracle.bc_dependencies(k * k, rowptr, np.array(cols, np.int32), 0)
    from math import comb
    for r in range(k):
        for c in range(k):
            assert depth[r * k + c] == r + c and sigma[r * k + c] == comb(r + c, r)
