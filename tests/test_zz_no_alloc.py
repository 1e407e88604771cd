"""pagerank_iter_noalloc (the entry point for callers that cannot allocate)
against pagerank_iter and the FP64 oracle: the same forms, two calls in a
row on one GPU with the second on a smaller graph (the static scratch keeps
the first call's contents), no allocation through the library's allocator
hook, and a refused oversize call that leaves its output untouched."""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.gpu_util import dev, host, load, torch

pytestmark = pytest.mark.gpu

L1_TOL = 1e-6
# (form, block width, merge range): plain forms, the stream-layout pull, the
# wide-block pull, the LDS push and the wide-block push
FORMS = [("plain_pull", 0, 0), ("plain_push", 0, 0), ("tocab_pull", 1 << 15, 16384),
         ("tocab_pull", 1 << 17, 1024), ("tocab_push", 1 << 13, 1024), ("tocab_push", 1 << 16, 1024)]


def l1(a, b):
    return float(np.abs(a.astype(np.float64) - b.astype(np.float64)).sum())


def _allocations():
    return torch().cuda.memory_stats().get("allocation.all.allocated", 0)


def _run(gc, g, h, form, W, k, iters):
    t = torch()
    part = None
    if form.startswith("tocab"):
        part = gc.tocab_partition(h, gc.GC_PULL if form == "tocab_pull" else gc.GC_PUSH, W, k)
    plain_dir = gc.GC_PUSH if form == "plain_push" else gc.GC_PULL
    rin = dev(np.full(g.n, 1.0 / g.n, np.float32))
    ref = t.empty(g.n, dtype=t.float32, device="cuda")
    out = t.full((g.n,), -1.0, dtype=t.float32, device="cuda")
    gc.pagerank_iter(h, part, plain_dir, 0.85, gc.GC_DANGLING_UNIFORM, rin, ref, iters)
    t.cuda.synchronize()
    before = _allocations()
    gc.pagerank_iter_noalloc(h, part, plain_dir, 0.85, gc.GC_DANGLING_UNIFORM, rin, out, iters)
    t.cuda.synchronize()
    assert _allocations() == before
    got, want = host(out), host(ref)
    if part is not None:
        part.free()
    return got, want


@pytest.mark.parametrize("form,W,k", FORMS, ids=lambda x: str(x))
def test_noalloc_matches_pagerank_iter_two_calls(form, W, k):
    import paper_1904_02241_amd as gc
    for g, iters in ((gg.rmat(16, 16, seed=1), 20), (gg.grid(150, 151, 0.05, seed=3), 9)):
        print(f"noalloc {form} W={W} k={k} n={g.n} m={g.m} iters={iters}", flush=True)
        h = load(g)
        got, want = _run(gc, g, h, form, W, k, iters)
        h.free()
        oracle_r = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, iters, mode=oracle.UNIFORM,
                                   r0=np.full(g.n, np.float64(np.float32(1.0 / g.n))))
        assert l1(got, want) <= L1_TOL
        assert l1(got, oracle_r) <= L1_TOL


def test_noalloc_refuses_more_than_its_scratch():
    """A plain push over 2^22 vertices needs 16 bytes per vertex, more than
    the 64 MiB of static scratch: GC_EINVAL, nothing queued, output intact."""
    import paper_1904_02241_amd as gc
    n = 1 << 22
    rowptr = np.arange(n + 1, dtype=np.int32)
    colidx = ((np.arange(n, dtype=np.int64) + 1) % n).astype(np.int32)  # one directed cycle
    h = gc.graph_load_csr(rowptr, colidx)
    t = torch()
    rin = t.full((n,), 1.0 / n, dtype=t.float32, device="cuda")
    out = t.full((n,), -1.0, dtype=t.float32, device="cuda")
    rc = gc.lib.pagerank_iter_noalloc(h.handle, None, gc.GC_PUSH, 0.85, gc.GC_DANGLING_UNIFORM,
                                      ctypes.c_void_p(rin.data_ptr()), ctypes.c_void_p(out.data_ptr()), 3, None)
    assert rc == gc.GC_EINVAL
    assert b"scratch" in gc.lib.gc_last_error()
    assert (host(out) == -1.0).all()
    # a plain pull of the same graph fits, and a cycle keeps every rank at 1/n
    gc.pagerank_iter_noalloc(h, None, gc.GC_PULL, 0.85, gc.GC_DANGLING_UNIFORM, rin, out, 3)
    np.testing.assert_allclose(host(out), 1.0 / n, rtol=1e-6)
    h.free()
