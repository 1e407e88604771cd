"""The comparison baselines of Section 4 (Base, VWC, conventional cache
blocking) against the FP64 oracle: L1 <= 1e-6 after 20 iterations."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.gpu_util import dev, host, load, torch

pytestmark = pytest.mark.gpu

L1_TOL = 1e-6


def ladder(gc, h, part, method, n, mode, iters=20):
    t = torch()
    rin = dev(np.full(n, 1.0 / n, np.float32))
    rout = t.empty(n, dtype=t.float32, device="cuda")
    gc.pagerank_ladder(h, part, method, 0.85, mode, rin, rout, iters)
    return host(rout), host(rin).astype(np.float64)


@pytest.mark.parametrize("method", ["BASE", "VWC", "VWC64", "CB"])
@pytest.mark.parametrize("mode", [oracle.UNIFORM, oracle.LEAK])
def test_ladder_rmat16_20_iterations(method, mode):
    import paper_1904_02241_amd as gc
    g = gg.rmat(16, 16, seed=1)
    h = load(g)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 12, 1024) if method == "CB" else None
    print(f"ladder rmat16 {method} mode={mode}", flush=True)
    got, r0 = ladder(gc, h, part, getattr(gc, f"GC_LADDER_{method}"), g.n, mode)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, mode=mode, r0=r0)
    err = float(np.abs(got.astype(np.float64) - want).sum())
    print(f"L1 = {err:.3e}")
    assert err <= L1_TOL
    if part is not None:
        part.free()
    h.free()


@pytest.mark.parametrize("W", [1 << 10, 1 << 13, 1 << 15, 1 << 18])
def test_ladder_cb_block_widths_on_ragged_grid(W):
    import paper_1904_02241_amd as gc
    g = gg.grid(300, 301, 0.05, seed=3)  # ragged last block
    h = load(g)
    part = gc.tocab_partition(h, gc.GC_PULL, W, 256)
    print(f"ladder grid CB W={W}", flush=True)
    got, r0 = ladder(gc, h, part, gc.GC_LADDER_CB, g.n, oracle.UNIFORM)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, r0=r0)
    assert float(np.abs(got.astype(np.float64) - want).sum()) <= L1_TOL
    part.free()
    h.free()


def test_ladder_rejects_bad_arguments():
    import paper_1904_02241_amd as gc
    g = gg.rmat(8, 8, seed=2)
    h = load(g)
    t = torch()
    rin = dev(np.full(g.n, 1.0 / g.n, np.float32))
    rout = t.empty(g.n, dtype=t.float32, device="cuda")
    with pytest.raises(gc.GraphCageError, match="unknown method"):
        gc.pagerank_ladder(h, None, 7, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, 1)
    with pytest.raises(gc.GraphCageError, match="GC_PULL partition"):
        gc.pagerank_ladder(h, None, gc.GC_LADDER_CB, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, 1)
    push = gc.tocab_partition(h, gc.GC_PUSH, 1 << 10, 256)
    with pytest.raises(gc.GraphCageError, match="GC_PULL partition"):
        gc.pagerank_ladder(h, push, gc.GC_LADDER_CB, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, 1)
    push.free()
    h.free()
