"""GPU PageRank until convergence (pagerank_converge) against the FP64 oracle.

The GPU measures the L1 change between its FP32 iterates and the oracle
between FP64 iterates, so the two may stop one iteration apart when a change
lies within rounding of the tolerance; the tolerance below is far above the
FP32 rounding of the change (about 1e-7), and every check is made against
the oracle run for the GPU's own number of iterations."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.gpu_util import dev, host, load, torch

pytestmark = pytest.mark.gpu

L1_TOL = 1e-6
FORMS = [("plain_pull", None, None), ("plain_push", None, None), ("tocab_pull", 1 << 15, 16384),
         ("tocab_pull", 1 << 12, 1024), ("tocab_pull", 1 << 18, 4096), ("tocab_push", 1 << 14, 4096)]


def run(gc, h, part, form, n, tol, max_iters, r0=None):
    t = torch()
    rin = dev(np.full(n, 1.0 / n, np.float32) if r0 is None else r0)
    rout = t.empty(n, dtype=t.float32, device="cuda")
    plain_dir = gc.GC_PUSH if form == "plain_push" else gc.GC_PULL
    k, delta = gc.pagerank_converge(h, part, plain_dir, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, tol, max_iters)
    return host(rout), k, delta, host(rin).astype(np.float64)


@pytest.mark.parametrize("form,W,K", FORMS, ids=lambda x: str(x))
def test_converge_rmat16_matches_oracle(form, W, K):
    import paper_1904_02241_amd as gc
    g = gg.rmat(16, 16, seed=1)
    h = load(g)
    part = None
    if form.startswith("tocab"):
        part = gc.tocab_partition(h, gc.GC_PULL if form == "tocab_pull" else gc.GC_PUSH, W, K)
    tol = 1e-4
    print(f"converge rmat16 {form} W={W} k={K}", flush=True)
    got, k, delta, r0 = run(gc, h, part, form, g.n, tol, 200)
    _, ko, deltas = oracle.pagerank_converge(g.n, g.rowptr, g.colidx, tol, 200, r0=r0)
    print(f"gpu {k} iterations delta {delta:.4e}; oracle {ko} iterations delta {deltas[-1]:.4e}", flush=True)
    assert abs(k - ko) <= 1 and delta <= tol
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, k, r0=r0)
    err = float(np.abs(got.astype(np.float64) - want).sum())
    print(f"L1 vs oracle iterate {k} = {err:.3e}")
    assert err <= L1_TOL
    # the reported change is the oracle's change at the same iteration (up to FP32 rounding of the iterates)
    _, _, deltas_k = oracle.pagerank_converge(g.n, g.rowptr, g.colidx, 0.0, k, r0=r0)
    assert abs(delta - deltas_k[k - 1]) <= 1e-6 + 1e-2 * delta
    if part is not None:
        part.free()
    h.free()


def test_converge_cycle_stops_after_one_iteration_and_cap_holds():
    import paper_1904_02241_amd as gc
    n = 4096
    rowptr = np.arange(n + 1, dtype=np.int32)
    colidx = ((np.arange(n) + 1) % n).astype(np.int32)
    h = gc.graph_load_csr(rowptr, colidx)
    got, k, delta, _ = run(gc, h, None, "plain_pull", n, 0.0, 50)
    assert (k, delta) == (1, 0.0)
    np.testing.assert_array_equal(got, np.full(n, np.float32(1.0 / n)))
    # max_iters caps a run that has not converged; rank_out holds that iterate
    g = gg.rmat(12, 8, seed=5)
    h2 = load(g)
    for cap in (1, 2, 7):
        got, k, delta, r0 = run(gc, h2, None, "plain_pull", g.n, 0.0, cap)
        assert k == cap and delta > 0.0
        want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, cap, r0=r0)
        assert float(np.abs(got.astype(np.float64) - want).sum()) <= L1_TOL
    h2.free()
    h.free()


def test_converge_rejects_bad_arguments():
    import paper_1904_02241_amd as gc
    g = gg.rmat(8, 8, seed=2)
    h = load(g)
    t = torch()
    rin = dev(np.full(g.n, 1.0 / g.n, np.float32))
    rout = t.empty(g.n, dtype=t.float32, device="cuda")
    for tol, cap in ((-1.0, 10), (float("nan"), 10), (1e-3, 0)):
        with pytest.raises(gc.GraphCageError, match="pagerank_converge"):
            gc.pagerank_converge(h, None, gc.GC_PULL, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, tol, cap)
    with pytest.raises(gc.GraphCageError, match="overlap"):
        gc.pagerank_converge(h, None, gc.GC_PULL, 0.85, gc.GC_DANGLING_UNIFORM, rin, rin, 1e-3, 10)
    h.free()
