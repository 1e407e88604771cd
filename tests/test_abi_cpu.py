"""C ABI checks that need no GPU: the library loads, exports every entry
point its header declares, and rejects bad arguments before queuing work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "graphcage.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while", "return")))


@pytest.fixture(scope="module")
def gc():
    import paper_1904_02241_amd as gc
    return gc


def test_header_lists_the_boundary():
    names = header_functions()
    for required in ("graph_load_csr", "tocab_partition", "pagerank_iter", "bfs_pull", "sssp_pull"):
        assert required in names


def test_library_exports_every_declared_symbol(gc):
    raw = ctypes.CDLL(gc.LIB_PATH)
    missing = [n for n in header_functions() if not hasattr(raw, n)]
    assert not missing, missing
    assert set(header_functions()) == set(gc.SIGNATURES)


def _status(fn, *args):
    return fn(*args)


def test_graph_load_rejects_bad_arguments(gc):
    out = ctypes.c_void_p()
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([1, 0], np.int32)
    L = gc.lib
    assert L.graph_load_csr(0, 0, rp.ctypes.data, ci.ctypes.data, None, 0, None, ctypes.byref(out)) == gc.GC_EINVAL
    assert "positive" in gc.gc_last_error()
    assert L.graph_load_csr(2, 2, None, ci.ctypes.data, None, 0, None, ctypes.byref(out)) == gc.GC_EINVAL
    assert L.graph_load_csr(2, 2, rp.ctypes.data, ci.ctypes.data, None, 0, None, None) == gc.GC_EINVAL
    assert L.graph_load_csr(2, 2, rp.ctypes.data, ci.ctypes.data, None, 0x10, None, ctypes.byref(out)) == gc.GC_EINVAL
    assert L.graph_load_csr(2, 1 << 31, rp.ctypes.data, ci.ctypes.data, None, 0, None,
                            ctypes.byref(out)) == gc.GC_EINVAL
    # rowptr[n] != m (host arrays are checked before anything is copied)
    assert L.graph_load_csr(2, 1, rp.ctypes.data, ci.ctypes.data, None, 0, None, ctypes.byref(out)) == gc.GC_EINVAL
    assert out.value is None


@pytest.mark.parametrize("rowptr,colidx,weight,needle", [
    ([0, 2, 1, 2], [1, 2], None, "decreases"),
    ([0, 1, 2], [1, 5], None, "out of range"),
    ([0, 1, 2], [0, 0], None, "self-loop"),
    ([0, 2, 2, 2], [2, 1], None, "ascending"),
    ([0, 2, 2, 2], [1, 1], None, "ascending"),
    ([0, 1, 2], [1, 0], [3, 0], "not positive"),
])
def test_validate_flag_catches_malformed_csr(gc, rowptr, colidx, weight, needle):
    out = ctypes.c_void_p()
    rp = np.array(rowptr, np.int32)
    ci = np.array(colidx, np.int32)
    w = None if weight is None else np.array(weight, np.int32)
    rc = gc.lib.graph_load_csr(len(rowptr) - 1, len(colidx), rp.ctypes.data, ci.ctypes.data,
                               None if w is None else w.ctypes.data, gc.GC_VALIDATE, None, ctypes.byref(out))
    assert rc == gc.GC_EINVAL
    assert needle in gc.gc_last_error()


def test_null_handles_rejected(gc):
    L = gc.lib
    out = ctypes.c_void_p()
    buf = np.zeros(8, np.float32)
    assert L.tocab_partition(None, gc.GC_PULL, 1 << 12, 0, None, ctypes.byref(out)) == gc.GC_EINVAL
    assert L.pagerank_iter(None, None, gc.GC_PULL, 0.85, 0, buf.ctypes.data, buf.ctypes.data, 1, None) == gc.GC_EINVAL
    assert L.bfs_pull(None, None, 0, buf.ctypes.data, None, 0, None) == gc.GC_EINVAL
    assert L.sssp_pull(None, None, 0, buf.ctypes.data, None, 0, None) == gc.GC_EINVAL
    assert L.graph_free(None) == gc.GC_EINVAL
    assert L.tocab_free(None) == gc.GC_EINVAL
    assert L.graph_info(None, None, None, None) == gc.GC_EINVAL
    assert L.tocab_info(None, None, None, None, None, None, None) == gc.GC_EINVAL
    assert L.graph_export_transpose(None, None, None, None, None) == gc.GC_EINVAL
    assert L.tocab_export(None, None, None, None, None, None, None, None) == gc.GC_EINVAL


def test_allocator_hook_needs_both_functions(gc):
    L = gc.lib
    assert L.gc_set_allocator(gc._torch_alloc, gc._FREE_FN(), None) == gc.GC_EINVAL
    assert "both" in gc.gc_last_error()
    assert L.gc_set_allocator(gc._torch_alloc, gc._torch_free, None) == gc.GC_OK


def test_import_fails_loudly_without_library(tmp_path):
    """The binding has no fallback: a missing library is an ImportError."""
    import subprocess
    import sys
    pkg = tmp_path / "paper_1904_02241_amd"
    pkg.mkdir()
    src = open(os.path.join(ROOT, "paper_1904_02241_amd", "__init__.py")).read()
    (pkg / "__init__.py").write_text(src)
    r = subprocess.run([sys.executable, "-c", "import paper_1904_02241_amd"], cwd=tmp_path,
                       capture_output=True, text=True)
    assert r.returncode != 0
    assert "is not built" in r.stderr
