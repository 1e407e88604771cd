"""GPU BFS / SSSP parity: depths and distances bit-exact against the oracle
(queue BFS, binary-heap Dijkstra) for every level policy and both pull
forms (plain and TOCAB)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import graphs
from tests.gpu_util import dev, host, load, torch

pytestmark = pytest.mark.gpu

GRAPHS = {
    "rmat16": lambda: gg.rmat(16, 16, seed=1),
    "rmat15_noperm": lambda: gg.rmat(15, 16, seed=2, permute=False),
    "grid300x301": lambda: gg.grid(300, 301, 0.05, seed=3),
    "grid_norewire": lambda: gg.grid(200, 190, 0.0, seed=3),
    "uniform": lambda: gg.uniform(70001, 200000, seed=4),
    "star_in": lambda: graphs.star_in(9000),
    "star_out": lambda: graphs.star_out(9000),
    "chain": lambda: graphs.chain(3000),
    "two_components": graphs.two_components,
    "dangling_mix": graphs.dangling_mix,
}

# (policy name, use a TOCAB partition)
VARIANTS = [("pull", False), ("pull", True), ("push", False), ("heuristic", False), ("heuristic", True)]


def _policy(gc, name):
    return {"pull": gc.GC_POLICY_PULL, "push": gc.GC_POLICY_PUSH, "heuristic": gc.GC_POLICY_HEURISTIC}[name]


def _sources(g, count=3):
    s = list(gg.sources(g, count, seed=21))
    return s + [0] if 0 not in s else s


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("policy,tocab", VARIANTS)
def test_bfs_bit_exact(name, policy, tocab):
    import paper_1904_02241_amd as gc
    g = GRAPHS[name]()
    print(f"bfs {name} {policy} tocab={tocab}", flush=True)
    h = load(g)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 10, 512) if tocab else None
    depth = torch().empty(g.n, dtype=torch().int32, device="cuda")
    for s in _sources(g):
        levels = gc.bfs_pull(h, part, s, depth, _policy(gc, policy))
        got = host(depth)
        want = oracle.bfs(g.n, g.rowptr, g.colidx, s)
        np.testing.assert_array_equal(got, want)
        assert levels == int(want[want != oracle.INF32].max()) + 1
    if part:
        part.free()
    h.free()


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("policy,tocab", VARIANTS)
def test_sssp_bit_exact(name, policy, tocab):
    import paper_1904_02241_amd as gc
    g = GRAPHS[name]().with_weights(31)
    print(f"sssp {name} {policy} tocab={tocab}", flush=True)
    h = load(g, weights=True)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 10, 1024) if tocab else None
    dist = torch().empty(g.n, dtype=torch().int32, device="cuda")
    for s in _sources(g):
        gc.sssp_pull(h, part, s, dist, _policy(gc, policy))
        got = host(dist)
        want = oracle.dijkstra(g.n, g.rowptr, g.colidx, g.weights, s)
        np.testing.assert_array_equal(got, want)
    if part:
        part.free()
    h.free()


@pytest.mark.parametrize("W,k", [(1 << 10, 1024), (1 << 15, 16384)])
def test_sssp_wide_weights_stream_layout(W, k):
    """Weights above 255 keep the int32 weight stream of the stream-layout
    SSSP pull (weights in [0, 255] are read as bytes); TOCAB pull and the
    heuristic stay bit-exact either way, and a path length past INT32_MAX is
    reported from the TOCAB pull as from the other forms."""
    import paper_1904_02241_amd as gc
    g = gg.rmat(14, 16, seed=12)
    rng = np.random.default_rng(5)
    g.weights = rng.integers(1, 100000, g.m, dtype=np.int32)
    h = load(g, weights=True)
    part = gc.tocab_partition(h, gc.GC_PULL, W, k)
    dist = torch().empty(g.n, dtype=torch().int32, device="cuda")
    for s in gg.sources(g, 3, seed=3):
        want = oracle.dijkstra(g.n, g.rowptr, g.colidx, g.weights, s)
        for pol in (gc.GC_POLICY_PULL, gc.GC_POLICY_HEURISTIC):
            gc.sssp_pull(h, part, int(s), dist, pol)
            np.testing.assert_array_equal(host(dist), want)
    part.free()
    h.free()
    c = graphs.chain(5)
    c.weights = np.full(c.m, 1 << 30, np.int32)
    hc = load(c, weights=True)
    pc = gc.tocab_partition(hc, gc.GC_PULL, 1 << 10, 1024)
    d = torch().empty(c.n, dtype=torch().int32, device="cuda")
    with pytest.raises(gc.GraphCageError) as e:
        gc.sssp_pull(hc, pc, 0, d, gc.GC_POLICY_PULL)
    assert e.value.code == gc.GC_EOVERFLOW
    pc.free()
    hc.free()


def test_bfs_equals_unit_weight_sssp():
    import paper_1904_02241_amd as gc
    g = gg.rmat(14, 16, seed=9)
    g.weights = np.ones(g.m, np.int32)
    h = load(g, weights=True)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 11, 2048)
    a = torch().empty(g.n, dtype=torch().int32, device="cuda")
    b = torch().empty_like(a)
    for s in gg.sources(g, 3, seed=1):
        gc.bfs_pull(h, part, s, a, gc.GC_POLICY_HEURISTIC)
        gc.sssp_pull(h, part, s, b, gc.GC_POLICY_HEURISTIC)
        np.testing.assert_array_equal(host(a), host(b))
    part.free()
    h.free()


def test_sssp_overflow_is_reported():
    import paper_1904_02241_amd as gc
    g = graphs.chain(5)
    g.weights = np.full(g.m, 1 << 30, np.int32)
    h = load(g, weights=True)
    dist = torch().empty(g.n, dtype=torch().int32, device="cuda")
    for policy in (gc.GC_POLICY_PULL, gc.GC_POLICY_PUSH):
        with pytest.raises(gc.GraphCageError) as e:
            gc.sssp_pull(h, None, 0, dist, policy)
        assert e.value.code == gc.GC_EOVERFLOW
    # a chain whose distances stay below INT32_MAX is fine
    g2 = graphs.chain(3)
    g2.weights = np.full(g2.m, 1 << 29, np.int32)
    h2 = load(g2, weights=True)
    d2 = torch().empty(g2.n, dtype=torch().int32, device="cuda")
    gc.sssp_pull(h2, None, 0, d2, gc.GC_POLICY_PULL)
    np.testing.assert_array_equal(host(d2), [0, 1 << 29, 1 << 30])
    h.free()
    h2.free()


def test_traversal_rejects_bad_arguments():
    import paper_1904_02241_amd as gc
    g = gg.rmat(10, 8, seed=1)
    h = load(g)
    d = torch().empty(g.n, dtype=torch().int32, device="cuda")
    with pytest.raises(gc.GraphCageError) as e:
        gc.sssp_pull(h, None, 0, d)  # unweighted
    assert e.value.code == gc.GC_EINVAL
    for bad in (-1, g.n):
        with pytest.raises(gc.GraphCageError):
            gc.bfs_pull(h, None, bad, d)
    push_part = gc.tocab_partition(h, gc.GC_PUSH, 1 << 10, 256)
    with pytest.raises(gc.GraphCageError):
        gc.bfs_pull(h, push_part, 0, d)
    with pytest.raises(gc.GraphCageError):
        gc.bfs_pull(h, None, 0, d, policy=7)
    host_buf = np.zeros(g.n, np.int32)
    with pytest.raises(gc.GraphCageError):
        gc.bfs_pull(h, None, 0, host_buf)
    push_part.free()
    h.free()


def test_isolated_source():
    import paper_1904_02241_amd as gc
    g = graphs.dangling_mix()  # vertex 5 has no arcs at all
    h = load(g.with_weights(3), weights=True)
    d = torch().empty(g.n, dtype=torch().int32, device="cuda")
    assert gc.bfs_pull(h, None, 5, d, gc.GC_POLICY_HEURISTIC) == 1
    want = np.full(g.n, oracle.INF32, np.int32)
    want[5] = 0
    np.testing.assert_array_equal(host(d), want)
    gc.sssp_pull(h, None, 5, d, gc.GC_POLICY_PULL)
    np.testing.assert_array_equal(host(d), want)
    h.free()


def test_heuristic_bfs_tocab_arm():
    """The working-set rule's BFS arm over a stream-layout partition: on a
    rewired grid (4 arcs per vertex) its dense middle pull levels run as
    TOCAB pull (trace action 2) and the late ones as plain pull; on R-MAT
    (16 arcs per vertex) no level runs as TOCAB. The level sequence on the
    grid follows the rule replayed on the host from the oracle's depths
    (direction-optimising test, then TOCAB while at least 1/64 of the arcs
    end at unvisited vertices). Depths stay bit-exact."""
    import paper_1904_02241_amd as gc
    cases = (("grid400", gg.grid(400, 400, 0.05, seed=3), True), ("rmat16", gg.rmat(16, 16, seed=1), False))
    for name, g, expect_tocab in cases:
        h = load(g)
        part = gc.tocab_partition(h, gc.GC_PULL, 1 << 12, 4096)
        assert gc.tocab_layout(part)["stream"]
        n, m = g.n, int(g.rowptr[-1])
        outd = np.diff(g.rowptr).astype(np.int64)
        ind = np.bincount(g.colidx, minlength=n).astype(np.int64)
        d = torch().empty(n, dtype=torch().int32, device="cuda")
        for s in gg.sources(g, 2, seed=21):
            print(f"heuristic bfs arm {name} source {s}", flush=True)
            gc.bfs_pull(h, part, int(s), d, gc.GC_POLICY_HEURISTIC)
            depth = host(d)
            want = oracle.bfs(n, g.rowptr, g.colidx, int(s))
            np.testing.assert_array_equal(depth, want)
            acts, _ = gc.traversal_trace(h)
            # the rule replayed from the oracle's levels
            exp, pulling = [], False
            m_u, m_u_in = m - int(outd[s]), m
            for lev in range(int(want[want != np.iinfo(np.int32).max].max()) + 1):
                fr = want == lev
                n_f, m_f = int(fr.sum()), int(outd[fr].sum())
                if not pulling and m_f > m_u / 14.0:
                    pulling = True
                elif pulling and n_f < n / 24.0:
                    pulling = False
                if not pulling:
                    exp.append(0)
                else:
                    exp.append(2 if (m <= 10 * n and m_u_in >= m / 64.0) else 1)
                nxt = want == lev + 1
                m_u -= int(outd[nxt].sum())
                m_u_in -= int(ind[nxt].sum())
            assert list(acts) == exp, (name, list(acts), exp)
            assert (2 in exp) == expect_tocab
        part.free()
        h.free()
