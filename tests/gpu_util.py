"""Helpers for the GPU parity tests (torch only moves memory)."""
import numpy as np


def torch():
    import torch as t
    return t


def dev(a):
    t = torch()
    return t.from_numpy(np.ascontiguousarray(a)).cuda()


def host(x):
    torch().cuda.synchronize()
    return x.cpu().numpy()


def load(g, weights=False):
    import paper_1904_02241_amd as gc
    return gc.graph_load_csr(g.rowptr, g.colidx, g.weights if weights else None)


def pagerank_gpu(gg_graph, form, mode, iters=20, W=1 << 10, k=256, r0=None, handles=None):
    """Runs one PageRank form through the C ABI; returns FP32 ranks (numpy)."""
    import paper_1904_02241_amd as gc
    t = torch()
    g = handles["g"] if handles else load(gg_graph)
    part = None
    if form.startswith("tocab"):
        d = gc.GC_PULL if form == "tocab_pull" else gc.GC_PUSH
        part = gc.tocab_partition(g, d, W, k)
    n = gg_graph.n
    rin = dev(np.full(n, 1.0 / n, np.float32) if r0 is None else r0.astype(np.float32))
    rout = t.empty(n, dtype=t.float32, device="cuda")
    plain_dir = gc.GC_PUSH if form == "plain_push" else gc.GC_PULL
    gc.pagerank_iter(g, part, plain_dir, 0.85, mode, rin, rout, iters)
    out = host(rout)
    r0_used = host(rin).astype(np.float64)
    if part is not None:
        part.free()
    if not handles:
        g.free()
    return out, r0_used
