"""GPU parity of the construction steps: transpose (graph_load_csr) and the
TOCAB partition, both bit-exact against the oracle."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import graphs
from tests.gpu_util import load

pytestmark = pytest.mark.gpu

GRAPHS = {
    "rmat16": lambda: gg.rmat(16, 16, seed=1),
    "rmat17_noperm": lambda: gg.rmat(17, 16, seed=2, permute=False),  # hub rows > 4096 arcs
    "grid300x301": lambda: gg.grid(300, 301, 0.05, seed=3),
    "uniform": lambda: gg.uniform(70001, 200000, seed=4),
    "dangling_mix": graphs.dangling_mix,
    "star_in": lambda: graphs.star_in(9000),  # one in-row of 8999 arcs
    "edgeless": lambda: graphs.edgeless(5),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_transpose_bit_exact(name):
    import paper_1904_02241_amd as gc
    g = GRAPHS[name]().with_weights(7)
    print(f"transpose {name} n={g.n} m={g.m}", flush=True)
    h = load(g, weights=True)
    tr = np.empty(g.n + 1, np.int32)
    tc = np.empty(max(g.m, 1), np.int32)
    tw = np.empty(max(g.m, 1), np.int32)
    gc.graph_export_transpose(h, tr, tc[:g.m] if g.m else tc, tw[:g.m] if g.m else tw)
    gc.gc_sync()
    h.free()
    wr, wc, ww = oracle.transpose(g.n, g.rowptr, g.colidx, g.weights)
    np.testing.assert_array_equal(tr, wr)
    np.testing.assert_array_equal(tc[:g.m], wc)
    np.testing.assert_array_equal(tw[:g.m], ww)


def export_partition(part, g):
    import paper_1904_02241_amd as gc
    info = part.info
    B, P, k = info["B"], info["P"], info["k"]
    R = -(-g.n // k)
    out = dict(blk_rowoff=np.empty(B + 1, np.int32), row_ptr=np.empty(P + 1, np.int32),
               id_map=np.empty(max(P, 1), np.int32), col=np.empty(max(g.m, 1), np.int32),
               w=np.empty(max(g.m, 1), np.int32), range_ptr=np.empty((R + 1) * B, np.int32))
    gc.tocab_export(part, out["blk_rowoff"], out["row_ptr"], out["id_map"], out["col"],
                    out["w"] if g.weights is not None else None, out["range_ptr"])
    gc.gc_sync()
    return out, B, P, R


@pytest.mark.parametrize("name", ["rmat16", "rmat17_noperm", "grid300x301", "uniform", "dangling_mix"])
@pytest.mark.parametrize("W,k", [(1 << 10, 256), (1 << 12, 4096), (1 << 14, 1024), (1 << 20, 16384)])
@pytest.mark.parametrize("direction", ["pull", "push"])
def test_partition_bit_exact(name, W, k, direction):
    import paper_1904_02241_amd as gc
    g = GRAPHS[name]().with_weights(9)
    print(f"partition {name} W={W} k={k} {direction}", flush=True)
    h = load(g, weights=True)
    d = gc.GC_PULL if direction == "pull" else gc.GC_PUSH
    part = gc.tocab_partition(h, d, W, k)
    got, B, P, R = export_partition(part, g)
    part.free()
    h.free()
    if direction == "pull":
        ar, ac, aw = oracle.transpose(g.n, g.rowptr, g.colidx, g.weights)
    else:
        ar, ac, aw = g.rowptr, g.colidx, g.weights
    want = oracle.partition(g.n, g.n, ar, ac, W, k, aw)
    assert (B, P) == (want.B, want.P)
    np.testing.assert_array_equal(got["blk_rowoff"], want.blk_rowoff)
    np.testing.assert_array_equal(got["row_ptr"], want.row_ptr)
    np.testing.assert_array_equal(got["id_map"][:P], want.id_map)
    np.testing.assert_array_equal(got["col"][:g.m], want.col)
    np.testing.assert_array_equal(got["w"][:g.m], want.w)
    np.testing.assert_array_equal(got["range_ptr"].reshape(R + 1, B).T, want.range_ptr)


def test_partition_rejects_bad_widths():
    import paper_1904_02241_amd as gc
    g = gg.rmat(12, 8, seed=1)
    h = load(g)
    for W, k in [(1000, 256), (1 << 9, 256), (1 << 12, 100), (1 << 12, 1 << 15)]:
        with pytest.raises(gc.GraphCageError) as e:
            gc.tocab_partition(h, gc.GC_PULL, W, k)
        assert e.value.code == gc.GC_EINVAL
    h.free()
