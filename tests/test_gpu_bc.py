"""GPU betweenness-centrality parity (Brandes' accumulation from a source
set) against the FP64 oracle, for every level policy and both pull forms.

Tolerance: path counts are integers summed in FP64 (exact below 2^53 in any
order); every dependency is a sum of positive terms, so a reordered sum
differs from the oracle's by at most about (levels x largest degree) units
of 2^-53 relative. rtol = 1e-9 leaves three orders of magnitude over that
for the graphs here (at most a few thousand arcs per vertex, at most a few
thousand levels on the chain whose dependencies are exact integers)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import graphs
from tests.gpu_util import dev, host, load, torch

pytestmark = pytest.mark.gpu

RTOL = 1e-9

GRAPHS = {
    "rmat14": lambda: gg.rmat(14, 16, seed=1),
    "rmat13_noperm": lambda: gg.rmat(13, 16, seed=2, permute=False),
    "grid120x121": lambda: gg.grid(120, 121, 0.05, seed=3),
    "uniform": lambda: gg.uniform(20001, 80000, seed=4),
    "star_in": lambda: graphs.star_in(5000),
    "star_out": lambda: graphs.star_out(5000),
    "chain": lambda: graphs.chain(1500),
    "two_components": graphs.two_components,
    "dangling_mix": graphs.dangling_mix,
    "dups_loops": graphs.with_dups_and_loops,
    "dense_level": lambda: _dense_level(60),
}


def _dense_level(k):
    """Source 0 -> 1..k (depth 1), every pair of 1..k joined both ways (arcs
    inside the level), 1 -> k + 1 and k + 1 -> k + 2 (depths 2, 3): the step
    of depth 1 has k(k - 1) + 1 out-arcs and the level below one in-arc, so
    the backward pushes there; the other steps pull."""
    src = [0] * k + [u for u in range(1, k + 1) for v in range(1, k + 1) if u != v] + [1, k + 1]
    dst = list(range(1, k + 1)) + [v for u in range(1, k + 1) for v in range(1, k + 1) if u != v] + [k + 1, k + 2]
    return gg.from_edges(k + 3, src, dst, name="dense_level")

# (policy name, use a TOCAB partition)
VARIANTS = [("pull", False), ("pull", True), ("push", False), ("heuristic", False), ("heuristic", True)]


def _policy(gc, name):
    return {"pull": gc.GC_POLICY_PULL, "push": gc.GC_POLICY_PUSH, "heuristic": gc.GC_POLICY_HEURISTIC}[name]


def _sources(g, count=3):
    s = [int(x) for x in gg.sources(g, count, seed=31)]
    return s + [0] if 0 not in s else s


def _check(got, want):
    scale = max(1.0, float(np.abs(want).max()))
    np.testing.assert_allclose(got, want, rtol=RTOL, atol=RTOL * scale)


@pytest.mark.parametrize("name", list(GRAPHS))
@pytest.mark.parametrize("policy,tocab", VARIANTS)
def test_bc_matches_oracle(name, policy, tocab):
    import paper_1904_02241_amd as gc
    g = GRAPHS[name]()
    print(f"bc {name} {policy} tocab={tocab}", flush=True)
    h = load(g)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 10, 512) if tocab else None
    srcs = _sources(g)
    bc = torch().zeros(g.n, dtype=torch().float64, device="cuda")
    gc.bc_accumulate(h, part, srcs, bc, _policy(gc, policy))
    _check(host(bc), oracle.bc(g.n, g.rowptr, g.colidx, srcs))
    if part:
        part.free()
    h.free()


@pytest.mark.parametrize("W,k", [(1 << 10, 256), (1 << 12, 2048), (1 << 15, 16384), (1 << 18, 4096)])
def test_bc_tocab_widths(W, k):
    """TOCAB forward levels over several block widths and merge ranges
    (several blocks and ranges, ragged last ones)."""
    import paper_1904_02241_amd as gc
    g = gg.rmat(15, 16, seed=5)
    print(f"bc rmat15 W={W} k={k}", flush=True)
    h = load(g)
    part = gc.tocab_partition(h, gc.GC_PULL, W, k)
    srcs = _sources(g, 2)
    bc = torch().zeros(g.n, dtype=torch().float64, device="cuda")
    gc.bc_accumulate(h, part, srcs, bc, gc.GC_POLICY_PULL)
    _check(host(bc), oracle.bc(g.n, g.rowptr, g.colidx, srcs))
    part.free()
    h.free()


def test_bc_accumulates_and_matches_single_sources():
    """bc is added into: two calls over disjoint source sets equal one call
    over their union, and the sum over single-source calls."""
    import paper_1904_02241_amd as gc
    g = gg.rmat(12, 16, seed=6)
    h = load(g)
    srcs = [int(x) for x in gg.sources(g, 4, seed=7)]
    one = torch().zeros(g.n, dtype=torch().float64, device="cuda")
    gc.bc_accumulate(h, None, srcs, one, gc.GC_POLICY_HEURISTIC)
    two = torch().zeros(g.n, dtype=torch().float64, device="cuda")
    gc.bc_accumulate(h, None, srcs[:2], two, gc.GC_POLICY_PUSH)
    gc.bc_accumulate(h, None, srcs[2:], two, gc.GC_POLICY_PULL)
    want = oracle.bc(g.n, g.rowptr, g.colidx, srcs)
    _check(host(one), want)
    _check(host(two), want)
    start = dev(np.full(g.n, 2.5))
    gc.bc_accumulate(h, None, srcs, start, gc.GC_POLICY_PULL)
    _check(host(start) - 2.5, want)
    h.free()


def test_bc_edge_cases():
    import paper_1904_02241_amd as gc
    # a source with no out-arcs, an empty source list, a repeated source
    g = graphs.dangling_mix()
    h = load(g)
    deg = np.diff(g.rowptr)
    sink = int(np.flatnonzero(deg == 0)[0])
    bc = torch().zeros(g.n, dtype=torch().float64, device="cuda")
    gc.bc_accumulate(h, None, [sink], bc, gc.GC_POLICY_HEURISTIC)
    gc.bc_accumulate(h, None, [], bc, gc.GC_POLICY_PULL)
    assert not host(bc).any()
    gc.bc_accumulate(h, None, [0, 0], bc, gc.GC_POLICY_PULL)
    _check(host(bc), oracle.bc(g.n, g.rowptr, g.colidx, [0, 0]))
    with pytest.raises(gc.GraphCageError):
        gc.bc_accumulate(h, None, [g.n], bc)
    with pytest.raises(gc.GraphCageError):
        gc.bc_accumulate(h, None, [0], bc, gc.GC_POLICY_LEARNED)
    with pytest.raises(gc.GraphCageError):
        gc.bc_accumulate(h, None, [0], host(bc))
    push = gc.tocab_partition(h, gc.GC_PUSH, 1 << 10, 256)
    with pytest.raises(gc.GraphCageError):
        gc.bc_accumulate(h, push, [0], bc)
    push.free()
    h.free()


def test_bc_rmat20_sampled_sources():
    """R-MAT scale 20 (the benchmark's graph family at 1/16 of its scale)
    from two sources, in the launch configuration the benchmark times."""
    import paper_1904_02241_amd as gc
    g = gg.rmat(20, 16, seed=8)
    print(f"bc rmat20 n={g.n} m={g.m}", flush=True)
    h = load(g)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 18, 4096)
    srcs = [int(x) for x in gg.sources(g, 2, seed=9)]
    want = oracle.bc(g.n, g.rowptr, g.colidx, srcs)
    for pol in (gc.GC_POLICY_HEURISTIC, gc.GC_POLICY_PULL):
        bc = torch().zeros(g.n, dtype=torch().float64, device="cuda")
        gc.bc_accumulate(h, part, srcs, bc, pol)
        _check(host(bc), want)
    part.free()
    h.free()
