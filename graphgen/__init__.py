"""Seeded synthetic graph inputs shared by the oracle and the GPU path.

Holds no arithmetic of the graph method itself: it only manufactures
out-edge CSR graphs (rows = source, columns ascending, no self-loops, no
duplicate arcs), arc weights, traversal sources and initial vectors.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        vp, i32, i64, u64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        lib.gg_rmat.restype = vp
        lib.gg_rmat.argtypes = [i32, i32, f64, f64, f64, u64, i32]
        lib.gg_grid.restype = vp
        lib.gg_grid.argtypes = [i32, i32, f64, u64]
        lib.gg_uniform.restype = vp
        lib.gg_uniform.argtypes = [i32, i64, u64]
        lib.gg_from_edges.restype = vp
        lib.gg_from_edges.argtypes = [i32, i64, vp, vp, i32]
        lib.gg_n.restype = i32
        lib.gg_n.argtypes = [vp]
        lib.gg_m.restype = i64
        lib.gg_m.argtypes = [vp]
        lib.gg_export.restype = None
        lib.gg_export.argtypes = [vp, vp, vp]
        lib.gg_free.restype = None
        lib.gg_free.argtypes = [vp]
        lib.gg_weights.restype = None
        lib.gg_weights.argtypes = [i32, vp, vp, u64, i32, vp]
        lib.gg_sources.restype = i32
        lib.gg_sources.argtypes = [i32, vp, u64, i32, vp]
        lib.gg_draw.restype = None
        lib.gg_draw.argtypes = [u64, i64, vp]
        lib.gg_threads.restype = i32
        _lib = lib
    return _lib


class Graph:
    """Out-edge CSR: rowptr int32[n+1], colidx int32[m]; optional int32 weights[m]."""

    def __init__(self, n, rowptr, colidx, weights=None, name="", undirected=False):
        self.n = int(n)
        self.m = int(colidx.shape[0])
        self.rowptr = rowptr
        self.colidx = colidx
        self.weights = weights
        self.name = name
        self.undirected = undirected

    def outdeg(self):
        return np.diff(self.rowptr).astype(np.int32)

    def with_weights(self, seed):
        w = np.empty(self.m, dtype=np.int32)
        _load().gg_weights(self.n, self.rowptr.ctypes.data, self.colidx.ctypes.data, seed,
                           1 if self.undirected else 0, w.ctypes.data)
        self.weights = w
        return self

    def __repr__(self):
        return f"Graph({self.name}, n={self.n}, m={self.m})"


def _take(h, name, undirected):
    if not h:
        raise ValueError(f"generator rejected its arguments ({name})")
    lib = _load()
    try:
        n, m = lib.gg_n(h), lib.gg_m(h)
        if m >= 2**31:
            raise ValueError("graph too large for int32 CSR")
        rowptr = np.empty(n + 1, dtype=np.int32)
        colidx = np.empty(m, dtype=np.int32)
        lib.gg_export(h, rowptr.ctypes.data, colidx.ctypes.data)
    finally:
        lib.gg_free(h)
    return Graph(n, rowptr, colidx, name=name, undirected=undirected)


def rmat(scale, edge_factor=16, seed=1, a=RMAT_A, b=RMAT_B, c=RMAT_C, permute=True):
    """Directed R-MAT graph, labels permuted by a seeded permutation."""
    h = _load().gg_rmat(scale, edge_factor, a, b, c, seed, 1 if permute else 0)
    return _take(h, f"rmat{scale}_ef{edge_factor}_s{seed}" + ("" if permute else "_noperm"), False)


def grid(rows=4096, cols=4096, p_rewire=0.05, seed=3):
    """Symmetric 4-neighbour lattice with a fraction of edges rewired."""
    h = _load().gg_grid(rows, cols, p_rewire, seed)
    return _take(h, f"grid{rows}x{cols}_p{p_rewire}_s{seed}", True)


def uniform(n, m_undirected, seed=4):
    """Symmetric uniform random graph with m_undirected generated edges."""
    h = _load().gg_uniform(n, m_undirected, seed)
    return _take(h, f"uniform_n{n}_m{m_undirected}_s{seed}", True)


def from_edges(n, src, dst, symmetrize=False, name="edges"):
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    assert src.shape == dst.shape
    h = _load().gg_from_edges(n, src.shape[0], src.ctypes.data, dst.ctypes.data, 1 if symmetrize else 0)
    return _take(h, name, bool(symmetrize))


def sources(g, count=8, seed=2):
    out = np.empty(count, dtype=np.int32)
    k = _load().gg_sources(g.n, g.rowptr.ctypes.data, seed, count, out.ctypes.data)
    return out[:k]


def draw(seed, count):
    out = np.empty(count, dtype=np.uint64)
    _load().gg_draw(seed, count, out.ctypes.data)
    return out


def threads():
    return _load().gg_threads()


def one_hot_seeds(g, count, seed):
    """Personalisation seed vertices (distinct, out-degree >= 1)."""
    return sources(g, count, seed)
