"""CPU oracle for GraphCage / TOCAB (Chen 2019). TEST INFRASTRUCTURE ONLY.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package. It shares no code with the GPU library: the plain C definitions
live in oracle.c (FP64 / int64, single-threaded) and this module only
marshals numpy arrays into them. Graphs are out-edge CSR (rowptr, colidx).
"""
import ctypes
import os

import numpy as np

from . import build as _build

INF32 = np.iinfo(np.int32).max
UNIFORM, LEAK = 0, 1

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        vp, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.oracle_pagerank.argtypes = [i32, vp, vp, f64, i32, i32, vp, vp]
        lib.oracle_ppr.argtypes = [i32, vp, vp, f64, i32, vp, vp]
        lib.oracle_bfs.argtypes = [i32, vp, vp, i32, vp]
        lib.oracle_dijkstra.argtypes = [i32, vp, vp, vp, i32, vp]
        lib.oracle_transpose.argtypes = [i32, vp, vp, vp, vp, vp, vp]
        lib.oracle_partition.argtypes = [i32, i32, vp, vp, vp, i32, i32, vp, vp,
                                         vp, vp, vp, vp, vp, vp]
        for f in ("oracle_pagerank", "oracle_ppr", "oracle_bfs", "oracle_dijkstra",
                  "oracle_transpose", "oracle_partition"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data


def pagerank(n, rowptr, colidx, d=0.85, iters=20, mode=UNIFORM, r0=None):
    """FP64 PageRank iterate `iters` from r0 (default uniform 1/n)."""
    rowptr, colidx = _i32(rowptr), _i32(colidx)
    r0 = np.full(n, 1.0 / n) if r0 is None else np.ascontiguousarray(r0, dtype=np.float64)
    out = np.empty(n, dtype=np.float64)
    rc = _load().oracle_pagerank(n, _ptr(rowptr), _ptr(colidx), d, mode, iters, _ptr(r0), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_pagerank rc={rc}")
    return out


def pagerank_converge(n, rowptr, colidx, tol, max_iters, d=0.85, mode=UNIFORM, r0=None):
    """FP64 PageRank run until the L1 change between consecutive iterates,
    sum_v |r_k[v] - r_{k-1}[v]|, is at most tol (Section 4 runs the methods
    until they converge; the test itself is not stated there, the L1 norm is
    the reading taken), or for max_iters iterations. One iteration is the
    plain definition above. Returns (r_k, k, [delta_1 .. delta_k])."""
    r = np.full(n, 1.0 / n) if r0 is None else np.ascontiguousarray(r0, dtype=np.float64)
    deltas = []
    for _ in range(max_iters):
        nxt = pagerank(n, rowptr, colidx, d, 1, mode, r0=r)
        deltas.append(float(np.abs(nxt - r).sum()))
        r = nxt
        if deltas[-1] <= tol:
            break
    return r, len(deltas), deltas


def spmv(n, rowptr, colidx, values, x):
    """FP64 sparse matrix-vector product over the out-arc CSR in the pull
    direction: y[v] = sum over arcs u -> v of values[arc] * x[u] (values
    None: every arc counts 1), accumulated in arc order."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    x = np.asarray(x, dtype=np.float64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    terms = x[src] if values is None else np.asarray(values, dtype=np.float64) * x[src]
    y = np.zeros(n, dtype=np.float64)
    np.add.at(y, colidx, terms)
    return y


def bc_dependencies(n, rowptr, colidx, source):
    """Brandes' single-source dependencies delta_s(v) over the out-arc CSR
    (unweighted shortest paths): a BFS from s counting shortest paths sigma
    level by level (a vertex at depth d+1 adds sigma of every in-neighbour at
    depth d, Algorithm 3's update), then, deepest level first,
    delta(v) = sum over arcs v -> w with depth(w) = depth(v) + 1 of
    sigma(v) / sigma(w) * (1 + delta(w)). FP64. Returns (delta, sigma, depth)
    with depth -1 for unreached vertices and delta(source) = 0."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    deg = np.diff(rowptr)
    depth = np.full(n, -1, dtype=np.int64)
    sigma = np.zeros(n, dtype=np.float64)
    depth[source], sigma[source] = 0, 1.0
    levels = [np.array([source], dtype=np.int64)]
    d = 0
    while True:
        f = levels[-1]
        src = np.repeat(f, deg[f])
        dst = colidx[np.concatenate([np.arange(rowptr[u], rowptr[u + 1]) for u in f])] if len(f) else f
        new = np.unique(dst[depth[dst] == -1])
        depth[new] = d + 1
        hit = depth[dst] == d + 1
        np.add.at(sigma, dst[hit], sigma[src[hit]])
        if len(new) == 0:
            break
        levels.append(new)
        d += 1
    delta = np.zeros(n, dtype=np.float64)
    for lv in range(len(levels) - 2, 0, -1):
        v = levels[lv]
        src = np.repeat(v, deg[v])
        w = colidx[np.concatenate([np.arange(rowptr[u], rowptr[u + 1]) for u in v])]
        hit = depth[w] == lv + 1
        np.add.at(delta, src[hit], sigma[src[hit]] / sigma[w[hit]] * (1.0 + delta[w[hit]]))
    return delta, sigma, depth


def bc(n, rowptr, colidx, sources):
    """Betweenness centrality restricted to the given sources:
    sum over s of delta_s(v) for v != s (FP64)."""
    out = np.zeros(n, dtype=np.float64)
    for s in sources:
        delta, _, _ = bc_dependencies(n, rowptr, colidx, int(s))
        delta[int(s)] = 0.0
        out += delta
    return out


def ppr(n, rowptr, colidx, p, d=0.85, iters=20):
    """FP64 personalised PageRank iterate `iters` from r0 = p."""
    rowptr, colidx = _i32(rowptr), _i32(colidx)
    p = np.ascontiguousarray(p, dtype=np.float64)
    out = np.empty(n, dtype=np.float64)
    rc = _load().oracle_ppr(n, _ptr(rowptr), _ptr(colidx), d, iters, _ptr(p), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_ppr rc={rc}")
    return out


def bfs(n, rowptr, colidx, source):
    rowptr, colidx = _i32(rowptr), _i32(colidx)
    out = np.empty(n, dtype=np.int32)
    rc = _load().oracle_bfs(n, _ptr(rowptr), _ptr(colidx), int(source), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_bfs rc={rc}")
    return out


def dijkstra(n, rowptr, colidx, weights, source):
    rowptr, colidx, weights = _i32(rowptr), _i32(colidx), _i32(weights)
    out = np.empty(n, dtype=np.int32)
    rc = _load().oracle_dijkstra(n, _ptr(rowptr), _ptr(colidx), _ptr(weights), int(source), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle_dijkstra rc={rc}")
    return out


def transpose(n, rowptr, colidx, weights=None):
    rowptr, colidx = _i32(rowptr), _i32(colidx)
    weights = None if weights is None else _i32(weights)
    t_rowptr = np.empty(n + 1, dtype=np.int32)
    t_colidx = np.empty(colidx.shape[0], dtype=np.int32)
    t_w = None if weights is None else np.empty(colidx.shape[0], dtype=np.int32)
    rc = _load().oracle_transpose(n, _ptr(rowptr), _ptr(colidx), _ptr(weights), _ptr(t_rowptr),
                                  _ptr(t_colidx), _ptr(t_w))
    if rc != 0:
        raise ValueError(f"oracle_transpose rc={rc}")
    return t_rowptr, t_colidx, t_w


class Partition:
    """Reference TOCAB partition (see oracle_partition in oracle.c)."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def partition(n_rows, n_cols, rowptr, colidx, W, k, weights=None):
    rowptr, colidx = _i32(rowptr), _i32(colidx)
    weights = None if weights is None else _i32(weights)
    lib = _load()
    B, P = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.oracle_partition(n_rows, n_cols, _ptr(rowptr), _ptr(colidx), _ptr(weights), W, k,
                              ctypes.byref(B), ctypes.byref(P), None, None, None, None, None, None)
    if rc != 0:
        raise ValueError(f"oracle_partition rc={rc}")
    B, P = B.value, P.value
    R = (n_rows + k - 1) // k
    m = colidx.shape[0]
    blk_rowoff = np.empty(B + 1, dtype=np.int64)
    row_ptr = np.empty(P + 1, dtype=np.int64)
    id_map = np.empty(P, dtype=np.int32)
    col = np.empty(m, dtype=np.int32)
    wout = None if weights is None else np.empty(m, dtype=np.int32)
    range_ptr = np.empty(B * (R + 1), dtype=np.int64)
    B2, P2 = ctypes.c_int64(), ctypes.c_int64()
    rc = lib.oracle_partition(n_rows, n_cols, _ptr(rowptr), _ptr(colidx), _ptr(weights), W, k,
                              ctypes.byref(B2), ctypes.byref(P2), _ptr(blk_rowoff), _ptr(row_ptr),
                              _ptr(id_map), _ptr(col), _ptr(wout), _ptr(range_ptr))
    if rc != 0:
        raise ValueError(f"oracle_partition rc={rc}")
    return Partition(B=B, P=P, R=R, W=W, k=k, blk_rowoff=blk_rowoff, row_ptr=row_ptr,
                     id_map=id_map, col=col, w=wout, range_ptr=range_ptr.reshape(B, R + 1))
