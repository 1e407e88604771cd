"""SpMV over the arcs in the pull direction (Section 4's SpMV benchmark),
plain and column-blocked, against the FP64 oracle. Products are FP32 and
sums FP64 on the GPU, so each y[v] is checked against the oracle within
4e-7 of the sum of the magnitudes of its terms (one FP32 rounding per
product and one of the result, plus FP64 summation). Blocks of at most 2^15
vertices run through the stream-layout pull, which sums inside a 512-arc
tile in FP32 (a lane's run of 8 arcs, a 6-step wave scan, the carried row
start) and stores the per-block partial in FP32: at most 17 FP32 roundings
on a row's way, so those widths get 20 * 2^-24 (1.2e-6) of the magnitude
sum."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests.gpu_util import dev, host, torch

pytestmark = pytest.mark.gpu


STREAM_MAX_W = 1 << 15


def tolerance(W):
    return 20 * 2.0 ** -24 if W is not None and W <= STREAM_MAX_W else 4e-7


def check(g, vals, x, y, rtol=4e-7):
    want = oracle.spmv(g.n, g.rowptr, g.colidx, vals, x)
    mag = oracle.spmv(g.n, g.rowptr, g.colidx, None if vals is None else np.abs(vals), np.abs(x))
    bad = np.abs(y.astype(np.float64) - want) > rtol * mag + 1e-30
    assert not bad.any(), f"{int(bad.sum())} entries off, first at {int(np.argmax(bad))}"


@pytest.mark.parametrize("values", ["f32", "int", "none"])
@pytest.mark.parametrize("W,K", [(None, None), (1 << 10, 256), (1 << 12, 4096), (1 << 15, 16384), (1 << 18, 512)],
                         ids=lambda v: str(v))
def test_spmv_rmat16(values, W, K):
    import paper_1904_02241_amd as gc
    g = gg.rmat(16, 16, seed=1)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1.0, 1.0, g.n).astype(np.float32)
    if values == "f32":
        vals = rng.uniform(-1.0, 1.0, g.m).astype(np.float32)
        h = gc.graph_load_csr(g.rowptr, g.colidx, values=vals)
    elif values == "int":
        vals = g.with_weights(11).weights
        h = gc.graph_load_csr(g.rowptr, g.colidx, vals)
    else:
        vals = None
        h = gc.graph_load_csr(g.rowptr, g.colidx)
    part = gc.tocab_partition(h, gc.GC_PULL, W, K) if W else None
    print(f"spmv rmat16 values={values} W={W} k={K}", flush=True)
    t = torch()
    xd = dev(x)
    y = t.empty(g.n, dtype=t.float32, device="cuda")
    gc.spmv(h, part, xd, y)
    check(g, None if vals is None else vals.astype(np.float64), x.astype(np.float64), host(y), tolerance(W))
    if part is not None:
        part.free()
    h.free()


def test_spmv_ragged_grid_and_isolated_vertices():
    import paper_1904_02241_amd as gc
    g = gg.grid(300, 301, 0.05, seed=3)
    rng = np.random.default_rng(8)
    vals = rng.uniform(0.5, 2.0, g.m).astype(np.float32)
    x = rng.uniform(0.0, 1.0, g.n).astype(np.float32)
    h = gc.graph_load_csr(g.rowptr, g.colidx, values=vals)
    t = torch()
    for W, K in ((None, None), (1 << 13, 256), (1 << 17, 1024)):
        part = gc.tocab_partition(h, gc.GC_PULL, W, K) if W else None
        y = t.full((g.n,), float("nan"), dtype=t.float32, device="cuda")
        gc.spmv(h, part, dev(x), y)
        check(g, vals.astype(np.float64), x.astype(np.float64), host(y), tolerance(W))  # no NaN left
        if part is not None:
            part.free()
    h.free()


def test_spmv_rejects_bad_arguments_and_sssp_refuses_values():
    import paper_1904_02241_amd as gc
    g = gg.rmat(8, 8, seed=2)
    vals = np.ones(g.m, np.float32)
    h = gc.graph_load_csr(g.rowptr, g.colidx, values=vals)
    t = torch()
    x = dev(np.ones(g.n, np.float32))
    with pytest.raises(gc.GraphCageError, match="overlap"):
        gc.spmv(h, None, x, x)
    push = gc.tocab_partition(h, gc.GC_PUSH, 1 << 10, 256)
    with pytest.raises(gc.GraphCageError, match="GC_PULL"):
        gc.spmv(h, push, x, t.empty(g.n, dtype=t.float32, device="cuda"))
    push.free()
    d = t.empty(g.n, dtype=t.int32, device="cuda")
    with pytest.raises(gc.GraphCageError, match="integer weights"):
        gc.sssp_pull(h, None, 0, d)
    h.free()


@pytest.mark.parametrize("values", ["f32", "int"])
def test_spmv_stream_layout_rmat20(values):
    """The stream-layout path at W = 2^15, k = 16384 (the benchmark's
    configuration at 1/16 of its scale; several chunks per block, the long
    hub rows that cross tiles), twice in a row (the padded value array is
    built by the first call)."""
    import paper_1904_02241_amd as gc
    g = gg.rmat(20, 16, seed=4)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1.0, 1.0, g.n).astype(np.float32)
    if values == "f32":
        vals = rng.uniform(0.0, 1.0, g.m).astype(np.float32)
        h = gc.graph_load_csr(g.rowptr, g.colidx, values=vals)
    else:
        vals = g.with_weights(13).weights
        h = gc.graph_load_csr(g.rowptr, g.colidx, vals)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 15, 16384)
    t = torch()
    for _ in range(2):
        y = t.full((g.n,), float("nan"), dtype=t.float32, device="cuda")
        gc.spmv(h, part, dev(x), y)
        check(g, vals.astype(np.float64), x.astype(np.float64), host(y), tolerance(1 << 15))
    part.free()
    h.free()
