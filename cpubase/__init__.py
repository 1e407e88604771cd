"""Multithreaded CPU performance baseline (OpenMP FP32 pull PageRank and
direction-optimising BFS on all host cores), timed beside the GPU path by
the benchmark. Not the oracle, and no part of the GPU library."""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _load():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "libcpubase.so")
        if not os.path.exists(path):
            raise ImportError("libcpubase.so is not built (run cpubase/build.py)")
        lib = ctypes.CDLL(path)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.cpub_threads.restype = ctypes.c_int
        lib.cpub_transpose.argtypes = [i32, i64, vp, vp, vp, vp]
        lib.cpub_transpose.restype = ctypes.c_int
        lib.cpub_pagerank_pull.argtypes = [i32, vp, vp, vp, ctypes.c_float, i32, vp]
        lib.cpub_pagerank_pull.restype = ctypes.c_double
        lib.cpub_bfs.argtypes = [i32, i64, vp, vp, vp, vp, i32, vp]
        lib.cpub_bfs.restype = ctypes.c_double
        _LIB = lib
    return _LIB


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def threads():
    return _load().cpub_threads()


class Graph:
    """Out-arc CSR plus the baseline's own in-arc CSR (built on construction)."""

    def __init__(self, n, rowptr, colidx):
        self.n, self.m = int(n), int(len(colidx))
        self.rowptr, self.colidx = _i32(rowptr), _i32(colidx)
        self.t_rowptr = np.empty(self.n + 1, np.int32)
        self.t_colidx = np.empty(max(self.m, 1), np.int32)
        rc = _load().cpub_transpose(self.n, self.m, self.rowptr.ctypes.data, self.colidx.ctypes.data,
                                    self.t_rowptr.ctypes.data, self.t_colidx.ctypes.data)
        if rc != 0:
            raise MemoryError("cpub_transpose")

    def pagerank(self, iters, d=0.85):
        """(FP32 ranks after `iters` iterations from 1/n, seconds)."""
        r = np.empty(self.n, np.float32)
        s = _load().cpub_pagerank_pull(self.n, self.rowptr.ctypes.data, self.t_rowptr.ctypes.data,
                                       self.t_colidx.ctypes.data, d, iters, r.ctypes.data)
        if s < 0:
            raise MemoryError("cpub_pagerank_pull")
        return r, s

    def bfs(self, source):
        """(int32 depths, INT32_MAX when unreachable; seconds)."""
        dep = np.empty(self.n, np.int32)
        s = _load().cpub_bfs(self.n, self.m, self.rowptr.ctypes.data, self.colidx.ctypes.data,
                             self.t_rowptr.ctypes.data, self.t_colidx.ctypes.data, int(source), dep.ctypes.data)
        if s < 0:
            raise MemoryError("cpub_bfs")
        return dep, s
