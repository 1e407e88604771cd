"""GPU scheduler network and learned policy.

Network parity against the FP64 oracle (oracle/mlp.py): forward outputs,
loss and gradient (relative error <= 1e-4), and Adam training steps. Policy:
traversals steered by the network stay bit-exact, a network without finite
outputs falls back to the heuristic, and collected rows are consistent."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import mlp
from tests.gpu_util import dev, host, load, torch

pytestmark = pytest.mark.gpu


def batch(K, B, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 6)).astype(np.float32)
    T = rng.normal(size=(B, K)).astype(np.float32)
    M = (rng.random((B, K)) < 0.8).astype(np.float32)
    M[0, 0] = 1.0
    return X, T, M


def rel_err(a, b):
    return float(np.max(np.abs(a - b)) / max(1e-12, np.max(np.abs(b))))


@pytest.mark.parametrize("K,B", [(1, 1), (4, 37), (9, 300)])
def test_forward_matches_oracle(K, B):
    import paper_1904_02241_amd as gc
    theta = mlp.init_params(K, seed=K).astype(np.float32)
    X, _, _ = batch(K, B, seed=1)
    m = gc.sched_create(K, theta)
    y = torch().empty((B, K), dtype=torch().float32, device="cuda")
    gc.sched_forward(m, dev(X), y)
    want, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64), K)
    assert rel_err(host(y), want) <= 1e-5
    np.testing.assert_array_equal(gc.sched_get_params(m), theta)
    m.free()


@pytest.mark.parametrize("K,B,weighted", [(2, 5, False), (5, 64, False), (9, 513, False), (9, 200, True)])
def test_loss_and_gradient_match_oracle(K, B, weighted):
    import paper_1904_02241_amd as gc
    theta = mlp.init_params(K, seed=10 + K).astype(np.float32)
    X, T, M = batch(K, B, seed=K)
    if weighted:  # per-row weights, as the trainer uses them
        M = M * np.random.default_rng(K).uniform(0.1, 3.0, size=(B, 1)).astype(np.float32)
    m = gc.sched_create(K, theta)
    loss = torch().zeros(1, dtype=torch().float32, device="cuda")
    grad = torch().zeros(gc.sched_param_count(K), dtype=torch().float32, device="cuda")
    gc.sched_loss_grad(m, dev(X), dev(T), dev(M), loss, grad)
    th64 = theta.astype(np.float64)
    Y, cache = mlp.forward(th64, X.astype(np.float64), K)
    want_l = mlp.loss(Y, T.astype(np.float64), M.astype(np.float64))
    want_g = mlp.backward(th64, cache, Y, T.astype(np.float64), M.astype(np.float64), K)
    assert abs(float(host(loss)[0]) - want_l) <= 1e-4 * abs(want_l)
    assert rel_err(host(grad), want_g) <= 1e-4
    m.free()


def test_adam_training_matches_oracle():
    import paper_1904_02241_amd as gc
    K, B, steps, lr = 4, 128, 25, 3e-3
    theta = mlp.init_params(K, seed=7).astype(np.float32)
    X, T, M = batch(K, B, seed=8)
    m = gc.sched_create(K, theta)
    hist = torch().zeros(steps, dtype=torch().float32, device="cuda")
    gc.sched_train(m, dev(X), dev(T), dev(M), steps, lr, hist)
    got = gc.sched_get_params(m)
    want, want_hist = mlp.train(theta.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                                M.astype(np.float64), K, steps, lr)
    np.testing.assert_allclose(host(hist), want_hist, rtol=1e-4)
    assert np.max(np.abs(got - want)) <= 1e-4 * max(1.0, np.max(np.abs(want)))
    m.free()


def test_features_are_the_documented_transform():
    import paper_1904_02241_amd as gc
    # prior level: 0.25 ms over 50,000 frontier out-arcs = 5 ns per arc
    f = gc.sched_features(1 << 20, 16 << 20, 1000, 60000, 3, 0.25, 50000)
    want = [np.log1p(1000), np.log1p(60000), np.log1p(16.0), np.log2(4 + 1), 3 / 16, np.log1p(5.0)]
    np.testing.assert_allclose(f, want, rtol=1e-6)


def _trained_policy(gc, g, h, parts):
    srcs = gg.sources(g, 4, seed=3)
    f1, t1 = gc.sched_collect(h, parts, 0, srcs)
    f2, t2 = gc.sched_collect(h, parts, 1, srcs)
    X = np.concatenate([f1, f2])
    T = np.log(np.maximum(np.concatenate([t1, t2]), 1e-4)).astype(np.float32)
    K = 2 + len(parts)
    m = gc.sched_create(K, mlp.init_params(K, seed=1).astype(np.float32))
    gc.sched_train(m, dev(X), dev(T), dev(np.ones_like(T)), 300, 3e-3)
    return m, X, T


def test_collect_and_learned_policy_stay_exact():
    import paper_1904_02241_amd as gc
    g = gg.rmat(14, 16, seed=5).with_weights(3)
    h = load(g, weights=True)
    parts = [gc.tocab_partition(h, gc.GC_PULL, W, 1024) for W in (1 << 11, 1 << 13)]
    m, X, T = _trained_policy(gc, g, h, parts)
    assert X.shape[0] >= 8 and np.all(np.isfinite(T))
    # collected features equal the documented transform of the first level
    f0 = gc.sched_features(g.n, g.m, 1, int(np.diff(g.rowptr)[gg.sources(g, 4, seed=3)[0]]), 0, 0.0)
    np.testing.assert_allclose(X[0], f0, rtol=1e-6)
    gc.sched_attach(h, m, parts)
    d = torch().empty(g.n, dtype=torch().int32, device="cuda")
    for s in gg.sources(g, 3, seed=9):
        gc.bfs_pull(h, None, s, d, gc.GC_POLICY_LEARNED)
        np.testing.assert_array_equal(host(d), oracle.bfs(g.n, g.rowptr, g.colidx, s))
        acts, ms = gc.traversal_trace(h)
        assert len(acts) >= 1 and np.all((acts >= 0) & (acts < 4)) and np.all(ms > 0)
        gc.sssp_pull(h, None, s, d, gc.GC_POLICY_LEARNED)
        np.testing.assert_array_equal(host(d), oracle.dijkstra(g.n, g.rowptr, g.colidx, g.weights, s))
    gc.sched_attach(h, None)
    with pytest.raises(gc.GraphCageError):
        gc.bfs_pull(h, None, 0, d, gc.GC_POLICY_LEARNED)  # nothing attached
    m.free()
    for p in parts:
        p.free()
    h.free()


def test_network_without_finite_output_falls_back_to_heuristic():
    import paper_1904_02241_amd as gc
    g = gg.rmat(13, 16, seed=6)
    h = load(g)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 11, 1024)
    theta = np.full(gc.sched_param_count(3), np.nan, np.float32)
    m = gc.sched_create(3, theta)
    gc.sched_attach(h, m, [part])
    d = torch().empty(g.n, dtype=torch().int32, device="cuda")
    s = int(gg.sources(g, 1, seed=1)[0])
    gc.bfs_pull(h, part, s, d, gc.GC_POLICY_LEARNED)
    np.testing.assert_array_equal(host(d), oracle.bfs(g.n, g.rowptr, g.colidx, s))
    learned, _ = gc.traversal_trace(h)
    gc.bfs_pull(h, part, s, d, gc.GC_POLICY_HEURISTIC)
    heur, _ = gc.traversal_trace(h)
    np.testing.assert_array_equal(learned, heur)
    with pytest.raises(gc.GraphCageError):
        gc.sched_attach(h, m, [])  # 3 outputs need one partition
    m.free()
    part.free()
    h.free()


@pytest.mark.parametrize("target", [1, 2])
def test_device_decision_follows_the_network(target):
    """A network with zero weights whose last-layer biases put action
    `target` (1 plain pull, 2 TOCAB pull over the attached partition) far
    below the others: under the learned policy every pull level runs as
    `target` and every push level as the rule's push. The decision for each
    level after the first is made on the device, by the last work-group of
    the previous level's count. BFS levels are unique, so the direction of
    each level is the rule's run with the partition given; SSSP is checked
    level by level for {push, target}. Results stay exact."""
    import paper_1904_02241_amd as gc
    g = gg.rmat(13, 16, seed=6).with_weights(5)
    h = load(g, weights=True)
    part = gc.tocab_partition(h, gc.GC_PULL, 1 << 11, 1024)
    K = 3
    theta = np.zeros(gc.sched_param_count(K), np.float32)
    theta[-K + target] = -5.0  # b3[target]: the only nonzero parameter
    m = gc.sched_create(K, theta)
    gc.sched_attach(h, m, [part])  # the network of every kind
    d = torch().empty(g.n, dtype=torch().int32, device="cuda")
    for s in gg.sources(g, 2, seed=3):
        s = int(s)
        print(f"device decision target {target} source {s}", flush=True)
        gc.bfs_pull(h, part, s, d, gc.GC_POLICY_HEURISTIC)
        heur, _ = gc.traversal_trace(h)
        gc.bfs_pull(h, None, s, d, gc.GC_POLICY_LEARNED)
        learned, _ = gc.traversal_trace(h)
        np.testing.assert_array_equal(host(d), oracle.bfs(g.n, g.rowptr, g.colidx, s))
        assert np.any(heur != 0) and heur[0] == 0
        np.testing.assert_array_equal(learned, np.where(heur == 0, 0, target))
        gc.sssp_pull(h, None, s, d, gc.GC_POLICY_LEARNED)
        learned, _ = gc.traversal_trace(h)
        np.testing.assert_array_equal(host(d), oracle.dijkstra(g.n, g.rowptr, g.colidx, g.weights, s))
        assert set(learned.tolist()) == {0, target}, learned
    gc.sched_attach(h, None)
    m.free()
    part.free()
    h.free()


def _train(gc, X, T, K, steps=3000, seed=1):
    """A network trained on rows X (features) and T (ms per action): targets
    are log times over each row's fastest action, rows weighted by the square
    root of their best time."""
    Tms = np.maximum(T, 1e-4)
    best = Tms.min(axis=1)
    M = np.repeat(np.sqrt(best / best.mean())[:, None], K, axis=1).astype(np.float32)
    m = gc.sched_create(K, mlp.init_params(K, seed=seed).astype(np.float32))
    gc.sched_train(m, dev(X), dev(np.log(Tms / best[:, None]).astype(np.float32)), dev(M), steps, 3e-3)
    return m


def test_trained_network_gains_over_heuristic():
    """Trains one network per traversal kind on levels collected on R-MAT 16
    and R-MAT 22 (seed 1, 8 sources) and runs BFS and SSSP on R-MAT 22 of
    another seed under the learned policy, the working-set heuristic (TOCAB
    over the attached partition nearest the paper's 2^18 blocks) and
    always-pull. Timings are the best of three runs per source over four
    sources.

    The rule keeps the direction of every level; the network picks the form
    of pull levels. SSSP gains: its pull levels run over 2^15 blocks, whose
    distances sit in LDS, where the rule's 2^18 blocks leave them in L2.
    BFS cannot: its pull levels read a status bitmap that already fits in
    L2, so plain pull (the rule's form) is the fastest form on every pull
    level of the training rows, the network keeps it, and BFS pays only the
    decision kernel queued after every level (about 5 us, some 5 % of a
    BFS of this size). The bars: SSSP a gain (1.05), BFS that cost and
    nothing more (0.9)."""
    import time
    import paper_1904_02241_amd as gc
    widths = [1 << 15, 1 << 16, 1 << 18, 1 << 20]
    K = 2 + len(widths)
    rows = {0: ([], []), 1: ([], [])}
    for scale in (16, 22):
        g = gg.rmat(scale, 16, seed=1).with_weights(11)
        h = load(g, weights=True)
        parts = [gc.tocab_partition(h, gc.GC_PULL, W, 16384 if W <= (1 << 15) else 4096) for W in widths]
        srcs = gg.sources(g, 8, seed=2)
        for kind in (0, 1):
            f, t = gc.sched_collect(h, parts, kind, srcs)
            rows[kind][0].append(f)
            rows[kind][1].append(t)
        for p in parts:
            p.free()
        h.free()
    nets = {kind: _train(gc, np.concatenate(rows[kind][0]), np.concatenate(rows[kind][1]), K) for kind in (0, 1)}

    g = gg.rmat(22, 16, seed=8).with_weights(11)
    h = load(g, weights=True)
    parts = [gc.tocab_partition(h, gc.GC_PULL, W, 16384 if W <= (1 << 15) else 4096) for W in widths]
    gc.sched_attach(h, nets[0], parts)
    gc.sched_attach_kind(h, 1, nets[1])
    d = torch().empty(g.n, dtype=torch().int32, device="cuda")
    srcs = gg.sources(g, 4, seed=8)
    mid = parts[widths.index(1 << 18)]
    gains = {}
    for kind, fn in (("bfs", gc.bfs_pull), ("sssp", gc.sssp_pull)):
        fn(h, None, int(srcs[0]), d, gc.GC_POLICY_HEURISTIC)  # warm-up
        total = {}
        for name, pol, part in (("learned", gc.GC_POLICY_LEARNED, None), ("heuristic", gc.GC_POLICY_HEURISTIC, mid),
                                ("always_pull", gc.GC_POLICY_PULL, None)):
            ms = 0.0
            for s in srcs:
                best_ms = np.inf
                for _ in range(3):
                    torch().cuda.synchronize()
                    t0 = time.perf_counter()
                    fn(h, part, int(s), d, pol)
                    torch().cuda.synchronize()
                    best_ms = min(best_ms, (time.perf_counter() - t0) * 1e3)
                ms += best_ms
            total[name] = ms
        # the learned traversal's result is still the exact one
        s = int(srcs[-1])
        fn(h, None, s, d, gc.GC_POLICY_LEARNED)
        want = (oracle.bfs(g.n, g.rowptr, g.colidx, s) if kind == "bfs"
                else oracle.dijkstra(g.n, g.rowptr, g.colidx, g.weights, s))
        np.testing.assert_array_equal(host(d), want)
        gains[kind] = (total["heuristic"] / total["learned"], total["always_pull"] / total["learned"])
        print(f"{kind}: learned {total['learned']:.2f} ms, heuristic {total['heuristic']:.2f} ms, always pull "
              f"{total['always_pull']:.2f} ms -> gain {gains[kind][0]:.3f}x over the heuristic, "
              f"{gains[kind][1]:.3f}x over always-pull")
    gc.sched_attach(h, None)
    for m in nets.values():
        m.free()
    for p in parts:
        p.free()
    h.free()
    assert gains["sssp"][0] >= 1.05, gains
    assert gains["bfs"][0] >= 0.9, gains
    for kind, (vs_heur, vs_pull) in gains.items():
        assert vs_pull > 1.0, (kind, vs_pull)


def _pagerank_l1(g, got):
    r0 = np.full(g.n, 1.0 / g.n)
    want = oracle.pagerank(g.n, g.rowptr, g.colidx, 0.85, 20, mode=oracle.UNIFORM, r0=r0)
    return float(np.abs(got.astype(np.float64) - want).sum())


def test_learned_pagerank_form():
    """PageRank under the learned scheduler: rows collected on R-MAT 16 and
    20 (every form timed from the same ranks), network trained on them, then
    pagerank_learned on R-MAT 21. The form it picks gives ranks within L1
    1e-6 of the oracle after 20 iterations, and its time per iteration is no
    worse than that of the method without the network (the working-set
    rule's TOCAB pull at 2^18)."""
    import time
    import paper_1904_02241_amd as gc
    widths = [1 << 15, 1 << 16, 1 << 18, 1 << 20]
    K = 2 + len(widths)
    X, T = [], []
    for scale in (16, 20):
        g = gg.rmat(scale, 16, seed=1)
        h = load(g)
        parts = [gc.tocab_partition(h, gc.GC_PULL, W, 4096) for W in widths]
        f, t = gc.sched_collect_pagerank(h, parts, rows=3)
        assert f.shape == (3, 6) and t.shape == (3, K) and (t > 0).all()
        X.append(f)
        T.append(t)
        for p in parts:
            p.free()
        h.free()
    X = np.concatenate(X)
    Tms = np.maximum(np.concatenate(T), 1e-4)
    best = Tms.min(axis=1)
    M = np.ones_like(Tms, dtype=np.float32)
    m = gc.sched_create(K, mlp.init_params(K, seed=1).astype(np.float32))
    gc.sched_train(m, dev(X), dev(np.log(Tms / best[:, None]).astype(np.float32)), dev(M), 2000, 3e-3)

    g = gg.rmat(21, 16, seed=8)
    h = load(g)
    parts = [gc.tocab_partition(h, gc.GC_PULL, W, 4096) for W in widths]
    tt = torch()
    rin = tt.full((g.n,), 1.0 / g.n, dtype=tt.float32, device="cuda")
    rout = tt.empty_like(rin)
    with pytest.raises(gc.GraphCageError):  # no network attached
        gc.pagerank_learned(h, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, 1)
    gc.sched_attach(h, m, parts)
    a = gc.pagerank_learned(h, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, 20)
    assert 0 <= a < K
    err = _pagerank_l1(g, host(rout))
    assert err <= 1e-6, err

    def per_iter(fn):
        fn(2)
        tt.cuda.synchronize()
        t0 = time.perf_counter()
        fn(10)
        tt.cuda.synchronize()
        return (time.perf_counter() - t0) / 10

    fixed = [per_iter(lambda k: gc.pagerank_iter(h, None, gc.GC_PUSH, 0.85, 0, rin, rout, k)),
             per_iter(lambda k: gc.pagerank_iter(h, None, gc.GC_PULL, 0.85, 0, rin, rout, k))]
    fixed += [per_iter(lambda k, p=p: gc.pagerank_iter(h, p, gc.GC_PULL, 0.85, 0, rin, rout, k)) for p in parts]
    learned = per_iter(lambda k: gc.pagerank_learned(h, 0.85, 0, rin, rout, k))
    print(f"learned form {a}: {learned * 1e3:.3f} ms/iter; fixed forms (push, pull, TOCAB@{widths}): "
          f"{[round(x * 1e3, 3) for x in fixed]}")
    fallback = fixed[2 + widths.index(1 << 18)]
    print(f"gain over the working-set rule's form: {fallback / learned:.2f}x")
    # the network's picks are timed against the rule's form before one is
    # kept, so the learned form is never the slower one (here 2^15 blocks,
    # about 4x faster than the rule's 2^18)
    assert learned <= fallback

    # a network without finite outputs: the working-set rule (TOCAB pull over
    # the attached width nearest 2^18)
    nan_net = gc.sched_create(K, np.full(gc.sched_param_count(K), np.nan, np.float32))
    gc.sched_attach(h, nan_net, parts)
    a = gc.pagerank_learned(h, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, 20)
    assert a == 2 + widths.index(1 << 18)
    assert _pagerank_l1(g, host(rout)) <= 1e-6
    gc.sched_attach(h, None)
    nan_net.free()
    m.free()
    for p in parts:
        p.free()
    h.free()


def test_learned_pagerank_edges():
    """A network without finite outputs and no attached partition falls back
    to plain pull (action 1); sched_collect refuses an unknown kind; PageRank
    rows of a graph hold one time per action."""
    import paper_1904_02241_amd as gc
    g = gg.rmat(12, 16, seed=4)
    h = load(g)
    tt = torch()
    rin = tt.full((g.n,), 1.0 / g.n, dtype=tt.float32, device="cuda")
    rout = tt.empty_like(rin)
    nan_net = gc.sched_create(2, np.full(gc.sched_param_count(2), np.nan, np.float32))
    gc.sched_attach(h, nan_net, [])
    assert gc.pagerank_learned(h, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, 20) == 1
    assert _pagerank_l1(g, host(rout)) <= 1e-6
    gc.sched_attach(h, None)
    f, t = gc.sched_collect_pagerank(h, [], rows=2)
    assert f.shape == (2, 6) and t.shape == (2, 2) and (t > 0).all()
    # a PageRank row: an all-active level 1 whose prior time is the working-set
    # form's (plain pull here: no partition) time per iteration over m arcs
    np.testing.assert_allclose(f[0], gc.sched_features(g.n, g.m, g.n, g.m, 1, float(t[0][1]), g.m), rtol=1e-6)
    with pytest.raises(gc.GraphCageError):
        gc.sched_collect(h, [], 3, [0])
    # per-kind networks: refused before sched_attach, on a wrong kind or K;
    # a PageRank network attached for kind 2 decides pagerank_learned alone
    two = gc.sched_create(2, np.full(gc.sched_param_count(2), np.nan, np.float32))
    with pytest.raises(gc.GraphCageError):
        gc.sched_attach_kind(h, 2, two)
    gc.sched_attach(h, two, [])
    with pytest.raises(gc.GraphCageError):
        gc.sched_attach_kind(h, 3, two)
    three = gc.sched_create(3, np.zeros(gc.sched_param_count(3), np.float32))
    with pytest.raises(gc.GraphCageError):
        gc.sched_attach_kind(h, 0, three)
    gc.sched_attach_kind(h, 2, nan_net)
    assert gc.pagerank_learned(h, 0.85, gc.GC_DANGLING_UNIFORM, rin, rout, 3) == 1
    gc.sched_attach_kind(h, 2, None)
    gc.sched_attach(h, None)
    three.free()
    two.free()
    nan_net.free()
    h.free()
