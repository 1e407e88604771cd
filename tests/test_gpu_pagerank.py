"""GPU PageRank parity against the FP64 oracle: L1 <= 1e-6 after 20
iterations (plain pull, plain push, TOCAB pull, TOCAB push)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import graphs
from tests.gpu_util import load, pagerank_gpu

pytestmark = pytest.mark.gpu

L1_TOL = 1e-6
FORMS = ["plain_pull", "plain_push", "tocab_pull", "tocab_push"]


def l1(a, b):
    return float(np.abs(a.astype(np.float64) - b).sum())


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("mode", [oracle.UNIFORM, oracle.LEAK])
def test_pagerank_rmat16_20_iterations(form, mode):
    g = gg.rmat(16, 16, seed=1)
    print(f"pagerank rmat16 {form} mode={mode}", flush=True)
    got, r0 = pagerank_gpu(g, form, mode)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, mode=mode, r0=r0)
    err = l1(got, want)
    print(f"L1 = {err:.3e}")
    assert err <= L1_TOL
    if mode == oracle.UNIFORM:
        assert abs(got.astype(np.float64).sum() - 1.0) < 1e-5


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("W,k", [(1 << 10, 256), (1 << 12, 4096), (1 << 14, 16384), (1 << 15, 2048),
                                 (1 << 15, 16384), (1 << 13, 256), (1 << 17, 512)])
def test_pagerank_ragged_grid_block_shapes(form, W, k):
    g = gg.grid(300, 301, 0.05, seed=3)  # n = 90300: ragged last block and range
    print(f"pagerank grid {form} W={W} k={k}", flush=True)
    got, r0 = pagerank_gpu(g, form, oracle.UNIFORM, W=W, k=k)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, r0=r0)
    assert l1(got, want) <= L1_TOL


@pytest.mark.parametrize("g", graphs.all_small(), ids=lambda g: g.name)
@pytest.mark.parametrize("form", FORMS)
def test_pagerank_small_graphs(g, form):
    got, r0 = pagerank_gpu(g, form, oracle.UNIFORM, iters=7)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 7, r0=r0)
    assert l1(got, want) <= L1_TOL


@pytest.mark.parametrize("form", FORMS)
def test_pagerank_hub_rows_longer_than_a_tile(form):
    """In-rows of 8999 and 20000 arcs: the whole-work-group path of a pull
    tile, inside one block (W = 2^14 >= n) and split over blocks (W = 2^10)."""
    for g in (graphs.star_in(9000), graphs.star_in(20001)):
        for W in (1 << 14, 1 << 10, 1 << 16):
            got, r0 = pagerank_gpu(g, form, oracle.UNIFORM, iters=5, W=W, k=1024)
            want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 5, r0=r0)
            assert l1(got, want) <= L1_TOL


@pytest.mark.parametrize("form", FORMS)
def test_pagerank_zero_and_one_iteration_and_custom_start(form):
    g = gg.rmat(12, 16, seed=5)
    rng = np.random.default_rng(3)
    r0 = rng.random(g.n).astype(np.float32)
    r0 /= r0.sum()
    got0, used = pagerank_gpu(g, form, oracle.UNIFORM, iters=0, r0=r0)
    np.testing.assert_array_equal(got0, r0.astype(np.float32))
    got1, used = pagerank_gpu(g, form, oracle.UNIFORM, iters=1, r0=r0)
    want1 = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 1, r0=used)
    assert l1(got1, want1) <= L1_TOL


def test_pagerank_chained_calls_continue_the_iteration():
    """20 iterations in one call equal 5 calls of 4 (the state is the rank)."""
    import paper_1904_02241_amd as gc
    from tests.gpu_util import dev, host, torch
    g = gg.rmat(14, 16, seed=2)
    h = load(g)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 11, 1024)
    t = torch()
    a = dev(np.full(g.n, 1.0 / g.n, np.float32))
    b = t.empty_like(a)
    for _ in range(5):
        gc.pagerank_iter(h, part, gc.GC_PULL, 0.85, 0, a, b, 4)
        a, b = b, a
    got = host(a)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, r0=np.full(g.n, np.float32(1.0 / g.n), np.float64))
    assert l1(got, want) <= L1_TOL
    part.free()
    h.free()


def test_pagerank_rejects_overlap_and_bad_args():
    import paper_1904_02241_amd as gc
    from tests.gpu_util import torch
    t = torch()
    g = gg.rmat(10, 8, seed=1)
    h = load(g)
    buf = t.zeros(2 * g.n, dtype=t.float32, device="cuda")
    with pytest.raises(gc.GraphCageError):
        gc.pagerank_iter(h, None, gc.GC_PULL, 0.85, 0, buf[: g.n], buf[g.n // 2: g.n // 2 + g.n], 1)
    with pytest.raises(gc.GraphCageError):
        gc.pagerank_iter(h, None, gc.GC_PULL, 1.5, 0, buf[: g.n], buf[g.n:], 1)
    with pytest.raises(gc.GraphCageError):
        gc.pagerank_iter(h, None, 7, 0.85, 0, buf[: g.n], buf[g.n:], 1)
    h.free()


@pytest.mark.timeout(900)
def test_pagerank_rmat22_tocab_and_plain():
    g = gg.rmat(22, 16, seed=1)
    print(f"pagerank rmat22 n={g.n} m={g.m}", flush=True)
    want = None
    for form, W in [("tocab_pull", 1 << 18), ("plain_pull", 0), ("tocab_push", 1 << 18)]:
        got, r0 = pagerank_gpu(g, form, oracle.UNIFORM, W=max(W, 1 << 10), k=4096)
        if want is None:
            want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, r0=r0)
        err = l1(got, want)
        print(f"{form}: L1 = {err:.3e}", flush=True)
        assert err <= L1_TOL


def test_autotune_picks_a_valid_width_and_caches_it():
    import paper_1904_02241_amd as gc
    g = gg.rmat(16, 16, seed=1)
    h = load(g)
    W, k, ms = gc.tocab_autotune(h, gc.GC_PULL)
    assert W & (W - 1) == 0 and (1 << 12) <= W <= (1 << 16)
    assert k in (2048, 4096, 8192) and ms > 0
    assert gc.tocab_autotune(h, gc.GC_PULL) == (W, k, ms)  # cached for this graph
    part = gc.tocab_partition(h, gc.GC_PULL, 0, 0)  # width 0: autotuned
    assert (part.info["W"], part.info["k"]) == (W, k)
    got, r0 = pagerank_gpu(g, "tocab_pull", oracle.UNIFORM, handles={"g": h}, W=W, k=k)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, r0=r0)
    assert l1(got, want) <= L1_TOL
    part.free()
    h.free()
