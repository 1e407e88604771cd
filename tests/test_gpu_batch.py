"""Batched persistent form: PageRank of many graphs and personalised
PageRank of several seeds in one launch, against the FP64 oracle (L1 <=
1e-6 per graph / per seed after 20 iterations), plus HIP-graph replays."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from tests import graphs
from tests.gpu_util import dev, host, load, torch

pytestmark = pytest.mark.gpu
L1_TOL = 1e-6


def build_inputs():
    gs = [gg.rmat(10, 16, seed=101), gg.rmat(12, 16, seed=102), gg.grid(70, 90, 0.05, 3),
          gg.uniform(20001, 60000, seed=4), graphs.dangling_mix(), gg.rmat(13, 8, seed=103)]
    pg = gg.rmat(12, 16, seed=7)
    seeds = gg.sources(pg, 8, seed=5)
    return gs, pg, seeds


def check(gs, pg, seeds, b, rout, pout, iters=20):
    import paper_1904_02241_amd as gc
    assert gc.batch_status(b)
    r = host(rout) if rout is not None else None
    for i, g in enumerate(gs):
        o0, o1 = b.rank_offsets[i], b.rank_offsets[i + 1]
        want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, iters, r0=np.full(g.n, np.float32(1.0 / g.n), np.float64))
        err = float(np.abs(r[o0:o1].astype(np.float64) - want).sum())
        assert err <= L1_TOL, (i, err)
    if len(seeds):
        p = host(pout)
        for q, s in enumerate(seeds):
            pv = np.zeros(pg.n)
            pv[s] = 1.0
            want = oracle.ppr(pg.n, pg.rowptr, pg.colidx, pv, 0.85, iters)
            err = float(np.abs(p[:, q].astype(np.float64) - want).sum())
            assert err <= L1_TOL, (q, err)


def test_batch_pagerank_and_ppr_in_one_launch():
    import paper_1904_02241_amd as gc
    gs, pg, seeds = build_inputs()
    hs = [load(g) for g in gs]
    hp = load(pg)
    b = gc.batch_create(hs, [1 << 16] * len(gs), hp, seeds)
    total = int(b.rank_offsets[-1])
    rin = dev(np.concatenate([np.full(g.n, 1.0 / g.n, np.float32) for g in gs]))
    rout = torch().empty(total, dtype=torch().float32, device="cuda")
    pout = torch().empty((pg.n, len(seeds)), dtype=torch().float32, device="cuda")
    gc.batch_run(b, 0.85, 20, rin, rout, pout)
    check(gs, pg, seeds, b, rout, pout)
    b.free()
    for h in hs + [hp]:
        h.free()


def test_batch_graph_replays_match_eager():
    import paper_1904_02241_amd as gc
    gs, pg, seeds = build_inputs()
    hs = [load(g) for g in gs]
    hp = load(pg)
    b = gc.batch_create(hs, None, hp, seeds)  # widths autotuned
    assert all(w >= (1 << 16) for w in b.block_widths)
    total = int(b.rank_offsets[-1])
    rin = dev(np.concatenate([np.full(g.n, 1.0 / g.n, np.float32) for g in gs]))
    rout = torch().empty(total, dtype=torch().float32, device="cuda")
    pout = torch().empty((pg.n, len(seeds)), dtype=torch().float32, device="cuda")
    gc.batch_run(b, 0.85, 20, rin, rout, pout)
    assert gc.batch_status(b)
    eager_r, eager_p = host(rout).copy(), host(pout).copy()
    gc.batch_capture(b, 0.85, 20, rin, rout, pout)
    for rep in range(3):
        rout.zero_()
        pout.zero_()
        x = torch().randn(1 << 20, device="cuda")  # eager work between replays
        _ = (x * 2).sum().item()
        gc.batch_launch(b)
        assert gc.batch_status(b)
        np.testing.assert_array_equal(host(rout), eager_r)
        np.testing.assert_allclose(host(pout), eager_p, rtol=0, atol=1e-9)
    check(gs, pg, seeds, b, rout, pout)
    b.free()
    for h in hs + [hp]:
        h.free()


def test_batch_ppr_only_and_graphs_only():
    import paper_1904_02241_amd as gc
    gs, pg, seeds = build_inputs()
    hp = load(pg)
    b = gc.batch_create([], None, hp, seeds[:3])
    pout = torch().empty((pg.n, 3), dtype=torch().float32, device="cuda")
    gc.batch_run(b, 0.85, 20, None, None, pout)
    check([], pg, seeds[:3], b, None, pout)
    b.free()
    hs = [load(g) for g in gs[:2]]
    b = gc.batch_create(hs, [1 << 16, 1 << 16])
    rin = dev(np.concatenate([np.full(g.n, 1.0 / g.n, np.float32) for g in gs[:2]]))
    rout = torch().empty(int(b.rank_offsets[-1]), dtype=torch().float32, device="cuda")
    gc.batch_run(b, 0.85, 20, rin, rout, None)
    check(gs[:2], pg, [], b, rout, None)
    b.free()
    for h in hs + [hp]:
        h.free()


def test_batch_rejects_bad_arguments():
    import paper_1904_02241_amd as gc
    g = gg.rmat(10, 8, seed=1)
    h = load(g)
    with pytest.raises(gc.GraphCageError):
        gc.batch_create([], None, None, [])
    with pytest.raises(gc.GraphCageError):
        gc.batch_create([], None, h, list(range(65)))
    with pytest.raises(gc.GraphCageError):
        gc.batch_create([], None, h, [g.n])
    with pytest.raises(gc.GraphCageError):
        gc.batch_create([h], [1 << 12])  # LDS-resident widths are not batched
    h.free()
