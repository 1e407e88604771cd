"""Python binding of the GraphCage / TOCAB HIP library (libgraphcage.so).

Argument marshalling only: every step runs inside the library's HIP
kernels. The functions carry the C ABI's names (include/graphcage.h).
Device arrays are torch CUDA tensors (HIP on ROCm); host arrays are numpy
arrays. PyTorch provides device memory (its caching allocator is installed
as the library's allocator on import) and streams; it computes nothing.

Importing fails loudly when the built library is missing: there is no
fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgraphcage.so")

GC_OK, GC_EINVAL, GC_ENOMEM, GC_EHIP, GC_EUNSUPPORTED, GC_EOVERFLOW = 0, -1, -2, -3, -4, -5
GC_UNREACHED = np.iinfo(np.int32).max
GC_DEVICE_PTRS, GC_VALIDATE, GC_VALUES_F32 = 1, 2, 4
GC_PULL, GC_PUSH = 0, 1
GC_DANGLING_UNIFORM, GC_DANGLING_LEAK = 0, 1
GC_POLICY_PULL, GC_POLICY_PUSH, GC_POLICY_HEURISTIC, GC_POLICY_LEARNED = 0, 1, 2, 3
GC_LADDER_BASE, GC_LADDER_VWC, GC_LADDER_VWC64, GC_LADDER_CB = 0, 1, 2, 3
GC_SCHED_INPUTS, GC_SCHED_HIDDEN = 6, 64

# every exported entry point, with (restype, argtypes)
_vp, _i32, _i64, _u32, _f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float
_p_i32, _p_i64 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)
_ALLOC_FN = ctypes.CFUNCTYPE(_vp, ctypes.c_size_t, _vp, _vp)
_FREE_FN = ctypes.CFUNCTYPE(None, _vp, _vp, _vp)
SIGNATURES = {
    "gc_last_error": (ctypes.c_char_p, []),
    "gc_set_allocator": (ctypes.c_int, [_ALLOC_FN, _FREE_FN, _vp]),
    "graph_load_csr": (ctypes.c_int, [_i32, _i64, _vp, _vp, _vp, _u32, _vp, ctypes.POINTER(_vp)]),
    "graph_info": (ctypes.c_int, [_vp, _p_i32, _p_i64, _p_i32]),
    "graph_export_transpose": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "graph_free": (ctypes.c_int, [_vp]),
    "tocab_partition": (ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, ctypes.POINTER(_vp)]),
    "tocab_info": (ctypes.c_int, [_vp, _p_i32, _p_i64, _p_i32, _p_i32, _p_i32, _p_i64]),
    "tocab_layout": (ctypes.c_int, [_vp, _p_i32, _p_i32, _p_i64]),
    "tocab_autotune": (ctypes.c_int, [_vp, _i32, _p_i32, _p_i32, ctypes.POINTER(ctypes.c_float), _vp]),
    "tocab_export": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "tocab_free": (ctypes.c_int, [_vp]),
    "pagerank_iter": (ctypes.c_int, [_vp, _vp, _i32, _f32, _i32, _vp, _vp, _i32, _vp]),
    "pagerank_iter_noalloc": (ctypes.c_int, [_vp, _vp, _i32, _f32, _i32, _vp, _vp, _i32, _vp]),
    "spmv": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "pagerank_ladder": (ctypes.c_int, [_vp, _vp, _i32, _f32, _i32, _vp, _vp, _i32, _vp]),
    "pagerank_converge": (ctypes.c_int, [_vp, _vp, _i32, _f32, _i32, _vp, _vp, ctypes.c_double, _i32, _p_i32,
                                         ctypes.POINTER(ctypes.c_double), _vp]),
    "bfs_pull": (ctypes.c_int, [_vp, _vp, _i32, _vp, _p_i32, _u32, _vp]),
    "sssp_pull": (ctypes.c_int, [_vp, _vp, _i32, _vp, _p_i32, _u32, _vp]),
    "bc_accumulate": (ctypes.c_int, [_vp, _vp, _vp, _i32, _vp, _u32, _vp]),
    "gc_sync": (ctypes.c_int, [_vp]),
    "traversal_trace": (ctypes.c_int, [_vp, _vp, _vp, _i32, _p_i32]),
    "sched_param_count": (ctypes.c_int, [_i32, _p_i64]),
    "sched_create": (ctypes.c_int, [_i32, _vp, ctypes.POINTER(_vp)]),
    "sched_get_params": (ctypes.c_int, [_vp, _vp, _vp]),
    "sched_forward": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp]),
    "sched_loss_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    "sched_train": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i32, _i32, _f32, _vp, _vp]),
    "sched_free": (ctypes.c_int, [_vp]),
    "sched_features": (ctypes.c_int, [_i32, _i64, _i32, _i64, _i32, _f32, _i64, _vp]),
    "sched_collect": (ctypes.c_int, [_vp, _vp, _i32, _i32, _vp, _i32, _vp, _vp, _i32, _p_i32, _vp]),
    "sched_attach": (ctypes.c_int, [_vp, _vp, _vp, _i32]),
    "sched_attach_kind": (ctypes.c_int, [_vp, _i32, _vp]),
    "pagerank_learned": (ctypes.c_int, [_vp, _f32, _i32, _vp, _vp, _i32, _p_i32, _vp]),
    "batch_create": (ctypes.c_int, [_vp, _i32, _vp, _vp, _vp, _i32, _vp, ctypes.POINTER(_vp)]),
    "batch_info": (ctypes.c_int, [_vp, _vp, _vp, _p_i32, _p_i64]),
    "batch_run": (ctypes.c_int, [_vp, _f32, _i32, _vp, _vp, _vp, _vp]),
    "batch_capture": (ctypes.c_int, [_vp, _f32, _i32, _vp, _vp, _vp]),
    "batch_launch": (ctypes.c_int, [_vp, _vp]),
    "batch_status": (ctypes.c_int, [_vp, _vp, _p_i32]),
    "batch_free": (ctypes.c_int, [_vp]),
    "gc_profile": (ctypes.c_int, [_i32]),
    "gc_profile_count": (ctypes.c_int, [_p_i32]),
    "gc_profile_get": (ctypes.c_int, [_i32, ctypes.c_char_p, _i32, ctypes.POINTER(ctypes.c_double), _p_i64]),
}


class GraphCageError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_1904_02241_amd/build.py "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


_alloc_error = None  # last exception of the torch allocator hook


def _check(rc, what):
    global _alloc_error
    if rc != GC_OK:
        msg = f"{what}: {lib.gc_last_error().decode()}"
        if rc == GC_ENOMEM and _alloc_error:
            msg += f" ({_alloc_error})"
            _alloc_error = None
        raise GraphCageError(rc, msg)


# ---------------------------------------------------------------------------
# torch as the device allocator and stream provider

def _torch():
    import torch
    return torch


@_ALLOC_FN
def _torch_alloc(nbytes, stream, ctx):
    global _alloc_error
    try:
        torch = _torch()
        torch.cuda.init()
        return torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
    except Exception as e:  # reported by the failing call
        _alloc_error = f"{type(e).__name__}: {e}"
        return None


@_FREE_FN
def _torch_free(ptr, stream, ctx):
    _torch().cuda.caching_allocator_delete(int(ptr))


def use_torch_allocator(enable=True):
    """Route the library's own device buffers through torch's caching allocator."""
    if enable:
        _check(lib.gc_set_allocator(_torch_alloc, _torch_free, None), "gc_set_allocator")
    else:
        _check(lib.gc_set_allocator(_ALLOC_FN(), _FREE_FN(), None), "gc_set_allocator")


use_torch_allocator(True)


def _stream(stream):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def _ptr(x):
    """Device or host address of a torch tensor or numpy array (contiguous)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        assert x.flags["C_CONTIGUOUS"], "array must be contiguous"
        return x.ctypes.data
    assert x.is_contiguous(), "tensor must be contiguous"
    return x.data_ptr()


def _is_device(x):
    return not isinstance(x, np.ndarray) and x.is_cuda


# ---------------------------------------------------------------------------
# handles

class Graph:
    def __init__(self, handle, n, m, weighted):
        self.handle, self.n, self.m, self.weighted = handle, n, m, weighted

    def free(self):
        if self.handle:
            _check(lib.graph_free(self.handle), "graph_free")
            self.handle = None


class Tocab:
    def __init__(self, handle, graph):
        self.handle, self.graph = handle, graph
        self.info = tocab_info(self)
        self.info.update(tocab_layout(self))

    def free(self):
        if self.handle:
            _check(lib.tocab_free(self.handle), "tocab_free")
            self.handle = None


def _h(obj):
    return None if obj is None else obj.handle


# ---------------------------------------------------------------------------
# C ABI, one wrapper per entry point

def gc_last_error():
    return lib.gc_last_error().decode()


def gc_sync(stream=None):
    _check(lib.gc_sync(_stream(stream)), "gc_sync")


def graph_load_csr(rowptr, colidx, weight=None, validate=False, stream=None, values=None):
    """Out-arc CSR (numpy int32 arrays or CUDA int32 tensors) -> Graph.
    `values` (float32, instead of `weight`) loads FP32 arc values for spmv."""
    n = int(rowptr.shape[0]) - 1
    m = int(colidx.shape[0])
    f32 = values is not None
    if f32:
        if weight is not None:
            raise ValueError("pass either weight or values")
        if isinstance(values, np.ndarray):
            weight = np.ascontiguousarray(values, dtype=np.float32).view(np.int32)
        else:
            import torch
            weight = values.contiguous().view(torch.int32)
    dev = _is_device(rowptr)
    for a in (colidx, weight):
        if a is not None and _is_device(a) != dev:
            raise ValueError("rowptr, colidx and weight must all be host or all be device arrays")
    flags = (GC_DEVICE_PTRS if dev else 0) | (GC_VALIDATE if validate else 0) | (GC_VALUES_F32 if f32 else 0)
    out = ctypes.c_void_p()
    _check(lib.graph_load_csr(n, m, _ptr(rowptr), _ptr(colidx), _ptr(weight), flags, _stream(stream),
                              ctypes.byref(out)), "graph_load_csr")
    return Graph(out, n, m, weight is not None)


def graph_info(g):
    n, m, w = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
    _check(lib.graph_info(_h(g), ctypes.byref(n), ctypes.byref(m), ctypes.byref(w)), "graph_info")
    return n.value, m.value, bool(w.value)


def graph_export_transpose(g, t_rowptr, t_colidx, t_weight=None, stream=None):
    _check(lib.graph_export_transpose(_h(g), _ptr(t_rowptr), _ptr(t_colidx), _ptr(t_weight), _stream(stream)),
           "graph_export_transpose")


def graph_free(g):
    g.free()


def tocab_partition(g, direction, block_width, merge_range=0, stream=None):
    out = ctypes.c_void_p()
    _check(lib.tocab_partition(_h(g), direction, block_width, merge_range, _stream(stream), ctypes.byref(out)),
           "tocab_partition")
    return Tocab(out, g)


def tocab_autotune(g, direction, stream=None):
    """(block_width, merge_range, ms per PageRank iteration) chosen for g."""
    W, k, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
    _check(lib.tocab_autotune(_h(g), direction, ctypes.byref(W), ctypes.byref(k), ctypes.byref(ms), _stream(stream)),
           "tocab_autotune")
    return W.value, k.value, ms.value


def tocab_info(t):
    B, P, W, k, d, b = (ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                        ctypes.c_int64())
    _check(lib.tocab_info(_h(t), ctypes.byref(B), ctypes.byref(P), ctypes.byref(W), ctypes.byref(k), ctypes.byref(d),
                          ctypes.byref(b)), "tocab_info")
    return {"B": B.value, "P": P.value, "W": W.value, "k": k.value, "dir": d.value, "bytes": b.value}


def tocab_layout(t):
    """{"stream": bool, "chunks": int, "table_bytes": int} of a partition's pull layout."""
    st, ch, tb = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib.tocab_layout(_h(t), ctypes.byref(st), ctypes.byref(ch), ctypes.byref(tb)), "tocab_layout")
    return {"stream": bool(st.value), "chunks": ch.value, "table_bytes": tb.value}


def tocab_export(t, blk_rowoff, row_ptr, id_map, col, weight, range_ptr, stream=None):
    _check(lib.tocab_export(_h(t), _ptr(blk_rowoff), _ptr(row_ptr), _ptr(id_map), _ptr(col), _ptr(weight),
                            _ptr(range_ptr), _stream(stream)), "tocab_export")


def tocab_free(t):
    t.free()


def pagerank_iter(g, t, dir_if_plain, damping, dangling, rank_in, rank_out, iters, stream=None):
    _check(lib.pagerank_iter(_h(g), _h(t), dir_if_plain, damping, dangling, _ptr(rank_in), _ptr(rank_out), iters,
                             _stream(stream)), "pagerank_iter")


def pagerank_iter_noalloc(g, t, dir_if_plain, damping, dangling, rank_in, rank_out, iters, stream=None):
    _check(lib.pagerank_iter_noalloc(_h(g), _h(t), dir_if_plain, damping, dangling, _ptr(rank_in), _ptr(rank_out),
                                     iters, _stream(stream)), "pagerank_iter_noalloc")


def spmv(g, t, x, y, stream=None):
    _check(lib.spmv(_h(g), _h(t), _ptr(x), _ptr(y), _stream(stream)), "spmv")


def pagerank_ladder(g, t, method, damping, dangling, rank_in, rank_out, iters, stream=None):
    _check(lib.pagerank_ladder(_h(g), _h(t), method, damping, dangling, _ptr(rank_in), _ptr(rank_out), iters,
                               _stream(stream)), "pagerank_ladder")


def pagerank_converge(g, t, dir_if_plain, damping, dangling, rank_in, rank_out, tol, max_iters, stream=None):
    """Returns (iterations run, last L1 change)."""
    iters, delta = ctypes.c_int32(0), ctypes.c_double(0.0)
    _check(lib.pagerank_converge(_h(g), _h(t), dir_if_plain, damping, dangling, _ptr(rank_in), _ptr(rank_out),
                                 float(tol), int(max_iters), ctypes.byref(iters), ctypes.byref(delta),
                                 _stream(stream)), "pagerank_converge")
    return iters.value, delta.value


def bfs_pull(g, t, source, depth, policy=GC_POLICY_PULL, stream=None):
    """Returns the number of levels run."""
    levels = ctypes.c_int32(0)
    _check(lib.bfs_pull(_h(g), _h(t), int(source), _ptr(depth), ctypes.byref(levels), policy, _stream(stream)),
           "bfs_pull")
    return levels.value


def sssp_pull(g, t, source, dist, policy=GC_POLICY_PULL, stream=None):
    """Returns the number of rounds run."""
    rounds = ctypes.c_int32(0)
    _check(lib.sssp_pull(_h(g), _h(t), int(source), _ptr(dist), ctypes.byref(rounds), policy, _stream(stream)),
           "sssp_pull")
    return rounds.value


def bc_accumulate(g, t, sources, bc, policy=GC_POLICY_PULL, stream=None):
    """Adds the dependencies of every source in `sources` (host ints) into
    bc (device float64[n])."""
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int32).reshape(-1))
    _check(lib.bc_accumulate(_h(g), _h(t), src.ctypes.data if src.size else None, int(src.size), _ptr(bc), policy,
                             _stream(stream)), "bc_accumulate")


def gc_profile(enable):
    _check(lib.gc_profile(1 if enable else 0), "gc_profile")


def gc_profile_read():
    """{kernel name: (total ms, launches)} of the events recorded so far."""
    cnt = ctypes.c_int32()
    _check(lib.gc_profile_count(ctypes.byref(cnt)), "gc_profile_count")
    out = {}
    for i in range(cnt.value):
        name = ctypes.create_string_buffer(128)
        ms, nl = ctypes.c_double(), ctypes.c_int64()
        _check(lib.gc_profile_get(i, name, 128, ctypes.byref(ms), ctypes.byref(nl)), "gc_profile_get")
        out[name.value.decode()] = (ms.value, nl.value)
    return out


# ---------------------------------------------------------------------------
# learned level scheduler

def traversal_trace(g, max_levels=4096):
    """(actions, ms) of every level of the last bfs_pull / sssp_pull on g."""
    acts = np.zeros(max_levels, np.int32)
    ms = np.zeros(max_levels, np.float32)
    cnt = ctypes.c_int32()
    _check(lib.traversal_trace(_h(g), acts.ctypes.data, ms.ctypes.data, max_levels, ctypes.byref(cnt)),
           "traversal_trace")
    k = min(cnt.value, max_levels)
    return acts[:k], ms[:k]


def sched_param_count(n_actions):
    c = ctypes.c_int64()
    _check(lib.sched_param_count(n_actions, ctypes.byref(c)), "sched_param_count")
    return c.value


class Sched:
    def __init__(self, handle, n_actions):
        self.handle, self.n_actions = handle, n_actions

    def free(self):
        if self.handle:
            _check(lib.sched_free(self.handle), "sched_free")
            self.handle = None


def sched_init_params(n_actions, seed):
    """Initial network parameters drawn by the caller (He-style uniform
    weights, zero biases), in the layout sched_create expects."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((GC_SCHED_INPUTS, GC_SCHED_HIDDEN), (GC_SCHED_HIDDEN, GC_SCHED_HIDDEN),
                            (GC_SCHED_HIDDEN, n_actions)):
        bound = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-bound, bound, size=(fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def sched_create(n_actions, params):
    params = np.ascontiguousarray(params, dtype=np.float32)
    assert params.shape == (sched_param_count(n_actions),)
    out = ctypes.c_void_p()
    _check(lib.sched_create(n_actions, params.ctypes.data, ctypes.byref(out)), "sched_create")
    return Sched(out, n_actions)


def sched_get_params(m):
    out = np.empty(sched_param_count(m.n_actions), np.float32)
    _check(lib.sched_get_params(_h(m), out.ctypes.data, _stream(None)), "sched_get_params")
    gc_sync()
    return out


def sched_forward(m, x, y, stream=None):
    _check(lib.sched_forward(_h(m), _ptr(x), int(x.shape[0]), _ptr(y), _stream(stream)), "sched_forward")


def sched_loss_grad(m, x, t, mask, loss, grad, stream=None):
    _check(lib.sched_loss_grad(_h(m), _ptr(x), _ptr(t), _ptr(mask), int(x.shape[0]), _ptr(loss), _ptr(grad),
                               _stream(stream)), "sched_loss_grad")


def sched_train(m, x, t, mask, steps, lr, loss_hist=None, stream=None):
    _check(lib.sched_train(_h(m), _ptr(x), _ptr(t), _ptr(mask), int(x.shape[0]), steps, lr, _ptr(loss_hist),
                           _stream(stream)), "sched_train")


def sched_free(m):
    m.free()


def sched_features(n, m, frontier, frontier_arcs, level, prior_ms, prior_arcs=0):
    out = np.empty(GC_SCHED_INPUTS, np.float32)
    _check(lib.sched_features(n, m, frontier, frontier_arcs, level, prior_ms, prior_arcs, out.ctypes.data),
           "sched_features")
    return out


def _handles(parts):
    arr = (ctypes.c_void_p * max(1, len(parts)))()
    for i, p in enumerate(parts):
        arr[i] = p.handle.value if isinstance(p.handle, ctypes.c_void_p) else p.handle
    return arr


def sched_collect(g, parts, kind, sources, max_rows=100000, stream=None):
    """(features [rows, 6], times_ms [rows, 2 + len(parts)]) of every level."""
    K = 2 + len(parts)
    feats = np.zeros((max_rows, GC_SCHED_INPUTS), np.float32)
    times = np.zeros((max_rows, K), np.float32)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    rows = ctypes.c_int32()
    _check(lib.sched_collect(_h(g), _handles(parts), len(parts), kind, src.ctypes.data, src.shape[0],
                             feats.ctypes.data, times.ctypes.data, max_rows, ctypes.byref(rows), _stream(stream)),
           "sched_collect")
    return feats[:rows.value], times[:rows.value]


def sched_collect_pagerank(g, parts, rows=4, stream=None):
    """(features [rows, 6], times_ms [rows, 2 + len(parts)]) of PageRank
    iterations (sched_collect kind 2)."""
    K = 2 + len(parts)
    feats = np.zeros((rows, GC_SCHED_INPUTS), np.float32)
    times = np.zeros((rows, K), np.float32)
    got = ctypes.c_int32()
    _check(lib.sched_collect(_h(g), _handles(parts), len(parts), 2, None, rows, feats.ctypes.data, times.ctypes.data,
                             rows, ctypes.byref(got), _stream(stream)), "sched_collect")
    return feats[:got.value], times[:got.value]


def pagerank_learned(g, damping, dangling, rank_in, rank_out, iters, stream=None):
    """Runs PageRank in the form the attached network picks; returns the action."""
    action = ctypes.c_int32(-1)
    _check(lib.pagerank_learned(_h(g), damping, dangling, _ptr(rank_in), _ptr(rank_out), iters,
                                ctypes.byref(action), _stream(stream)), "pagerank_learned")
    return action.value


def sched_attach(g, m, parts=()):
    _check(lib.sched_attach(_h(g), _h(m), _handles(parts) if m is not None else None,
                            len(parts) if m is not None else 0), "sched_attach")


def sched_attach_kind(g, kind, m):
    """Network m for one kind of work only (0 BFS, 1 SSSP, 2 PageRank), over the
    partitions of the last sched_attach; None returns the kind to the shared one."""
    _check(lib.sched_attach_kind(_h(g), int(kind), _h(m)), "sched_attach_kind")


# ---------------------------------------------------------------------------
# batched persistent form

class Batch:
    def __init__(self, handle, graphs, n_seeds):
        self.handle, self.graphs, self.n_seeds = handle, graphs, n_seeds
        G = len(graphs)
        offs = np.zeros(G + 1, np.int64)
        widths = np.zeros(max(G, 1), np.int32)
        grid, nbytes = ctypes.c_int32(), ctypes.c_int64()
        _check(lib.batch_info(handle, offs.ctypes.data, widths.ctypes.data, ctypes.byref(grid), ctypes.byref(nbytes)),
               "batch_info")
        self.rank_offsets, self.block_widths, self.grid, self.bytes = offs, widths[:G], grid.value, nbytes.value

    def free(self):
        if self.handle:
            _check(lib.batch_free(self.handle), "batch_free")
            self.handle = None


def batch_create(graphs, block_widths=None, ppr_graph=None, seeds=(), stream=None):
    G = len(graphs)
    hs = _handles(graphs)
    w = None if block_widths is None else np.ascontiguousarray(block_widths, np.int32)
    sd = np.ascontiguousarray(seeds, np.int32)
    out = ctypes.c_void_p()
    _check(lib.batch_create(hs if G else None, G, None if w is None else w.ctypes.data, _h(ppr_graph),
                            sd.ctypes.data if len(sd) else None, len(sd), _stream(stream), ctypes.byref(out)),
           "batch_create")
    return Batch(out, list(graphs), len(sd))


def batch_run(b, damping, iters, ranks_in, ranks_out, ppr_out, stream=None):
    _check(lib.batch_run(_h(b), damping, iters, _ptr(ranks_in), _ptr(ranks_out), _ptr(ppr_out), _stream(stream)),
           "batch_run")


def batch_capture(b, damping, iters, ranks_in, ranks_out, ppr_out):
    _check(lib.batch_capture(_h(b), damping, iters, _ptr(ranks_in), _ptr(ranks_out), _ptr(ppr_out)), "batch_capture")


def batch_launch(b, stream=None):
    _check(lib.batch_launch(_h(b), _stream(stream)), "batch_launch")


def batch_status(b, stream=None):
    """True when the last launch finished without a barrier time-out."""
    flag = ctypes.c_int32()
    _check(lib.batch_status(_h(b), _stream(stream), ctypes.byref(flag)), "batch_status")
    return flag.value == 0


def batch_free(b):
    b.free()
