"""Parity in the configurations the benchmark suites time, beside the
smaller cases of the other test files.

* Batched form as benchmarked: 32 R-MAT graphs (scales 14-20, edge factor
  16, seeds 100-131) with autotuned block widths plus 64 personalised
  PageRank seeds on R-MAT 22, 20 iterations in one graph-replayed launch.
  Every graph's ranks are checked (L1 <= 1e-6 against the FP64 oracle), and
  PPR lanes 0, 31 and 63 on R-MAT 22; all 64 lanes are checked on R-MAT 18.
* Betweenness centrality and SpMV through the wide-block partition the
  benchmark uses (W = 2^18, merge range k = 4096, several blocks).

The oracle is single-threaded per call; independent oracle calls run in a
thread pool (the C oracle releases the interpreter lock)."""
import concurrent.futures
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.gpu_util import dev, host, load, torch

pytestmark = pytest.mark.gpu
L1_TOL = 1e-6
C4_SCALES = [14] * 5 + [15] * 5 + [16] * 5 + [17] * 5 + [18] * 4 + [19] * 4 + [20] * 4


def _pool():
    return concurrent.futures.ThreadPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1)))


def _pagerank_want(g):
    return oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, r0=np.full(g.n, np.float32(1.0 / g.n), np.float64))


def _ppr_want(g, s):
    p = np.zeros(g.n)
    p[s] = 1.0
    return oracle.ppr(g.n, g.rowptr, g.colidx, p, 0.85, 20)


@pytest.mark.timeout(900)
def test_c4_batch_as_benchmarked():
    import paper_1904_02241_amd as gc
    t = torch()
    ghs = [gg.rmat(sc, 16, seed=100 + i) for i, sc in enumerate(C4_SCALES)]
    pgh = gg.rmat(22, 16, seed=6)
    seeds = gg.sources(pgh, 64, seed=7)
    lanes = [0, 31, 63]
    with _pool() as ex:
        fut_g = [ex.submit(_pagerank_want, x) for x in ghs]
        fut_p = [ex.submit(_ppr_want, pgh, int(seeds[q])) for q in lanes]
        hs = [load(x) for x in ghs]
        hp = load(pgh)
        b = gc.batch_create(hs, None, hp, seeds)
        print(f"c4 batch widths {list(b.block_widths)} grid {b.grid}", flush=True)
        rin = t.cat([t.full((x.n,), 1.0 / x.n, dtype=t.float32, device="cuda") for x in ghs])
        rout = t.empty_like(rin)
        pout = t.empty((pgh.n, 64), dtype=t.float32, device="cuda")
        gc.batch_capture(b, 0.85, 20, rin, rout, pout)
        gc.batch_launch(b)
        assert gc.batch_status(b)
        r, p = host(rout), host(pout)
        for i, x in enumerate(ghs):
            o0, o1 = b.rank_offsets[i], b.rank_offsets[i + 1]
            err = float(np.abs(r[o0:o1].astype(np.float64) - fut_g[i].result()).sum())
            print(f"graph {i} rmat{C4_SCALES[i]} W={b.block_widths[i]} L1 = {err:.3e}", flush=True)
            assert err <= L1_TOL, (i, err)
        for q, f in zip(lanes, fut_p):
            err = float(np.abs(p[:, q].astype(np.float64) - f.result()).sum())
            print(f"ppr rmat22 lane {q} seed {int(seeds[q])} L1 = {err:.3e}", flush=True)
            assert err <= L1_TOL, (q, err)
    b.free()
    for h in hs + [hp]:
        h.free()


@pytest.mark.timeout(600)
def test_ppr_all_64_lanes_rmat18():
    import paper_1904_02241_amd as gc
    t = torch()
    pgh = gg.rmat(18, 16, seed=6)
    seeds = gg.sources(pgh, 64, seed=7)
    with _pool() as ex:
        futs = [ex.submit(_ppr_want, pgh, int(s)) for s in seeds]
        hp = load(pgh)
        b = gc.batch_create([], None, hp, seeds)
        pout = t.empty((pgh.n, 64), dtype=t.float32, device="cuda")
        gc.batch_run(b, 0.85, 20, None, None, pout)
        assert gc.batch_status(b)
        p = host(pout)
        worst = 0.0
        for q, f in enumerate(futs):
            err = float(np.abs(p[:, q].astype(np.float64) - f.result()).sum())
            worst = max(worst, err)
            assert err <= L1_TOL, (q, err)
        print(f"ppr rmat18, 64 lanes: worst L1 = {worst:.3e}", flush=True)
    b.free()
    hp.free()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("policy", ["pull", "heuristic"])
def test_bc_wide_blocks_k4096(policy):
    """W = 2^18, k = 4096 over R-MAT 20 (B = 4 blocks): the merge the
    benchmark's BC suite runs (flattened slices, 4096-vertex ranges)."""
    import paper_1904_02241_amd as gc
    g = gg.rmat(20, 16, seed=1)
    srcs = [int(x) for x in gg.sources(g, 2, seed=5)]
    h = load(g)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 18, 4096)
    assert part.info["B"] == 4
    bc = torch().zeros(g.n, dtype=torch().float64, device="cuda")
    pol = gc.GC_POLICY_PULL if policy == "pull" else gc.GC_POLICY_HEURISTIC
    gc.bc_accumulate(h, part, srcs, bc, pol)
    want = oracle.bc(g.n, g.rowptr, g.colidx, srcs)
    got = host(bc)
    scale = max(1.0, float(np.abs(want).max()))
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-9 * scale)
    part.free()
    h.free()


@pytest.mark.timeout(600)
def test_spmv_wide_blocks_k4096():
    """SpMV through the tile kernel and the flattened k = 4096 merge (W =
    2^18 over R-MAT 20, B = 4), FP32 arc values: every y[v] within 4e-7 of
    the sum of its terms' magnitudes (FP32 products and result, FP64 sums)."""
    import paper_1904_02241_amd as gc
    g = gg.rmat(20, 16, seed=1)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1.0, 1.0, g.n).astype(np.float32)
    vals = rng.uniform(-1.0, 1.0, g.m).astype(np.float32)
    h = gc.graph_load_csr(g.rowptr, g.colidx, values=vals)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 18, 4096)
    assert part.info["B"] == 4
    y = torch().empty(g.n, dtype=torch().float32, device="cuda")
    gc.spmv(h, part, dev(x), y)
    got = host(y).astype(np.float64)
    want = oracle.spmv(g.n, g.rowptr, g.colidx, vals.astype(np.float64), x.astype(np.float64))
    mag = oracle.spmv(g.n, g.rowptr, g.colidx, np.abs(vals.astype(np.float64)), np.abs(x.astype(np.float64)))
    bad = np.abs(got - want) > 4e-7 * mag + 1e-30
    assert not bad.any(), f"{int(bad.sum())} entries off"
    part.free()
    h.free()
