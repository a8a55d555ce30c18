"""The C-ABI library loads, exports every symbol bfs.h declares, and rejects bad
arguments before touching a device (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1604_02844_amd as bfs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "bfs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(bfs_[a-z_0-9]+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = bfs.load_library()
    names = declared_functions()
    assert len(names) >= 14, names
    for name in names:
        assert hasattr(lib, name), f"libbfs.so does not export {name}"
    assert set(bfs.ABI_SYMBOLS) <= set(names)


def test_status_strings():
    for code, name in [(0, "BFS_OK"), (1, "BFS_PENDING"), (-1, "BFS_E_INVALID_ARG"), (-2, "BFS_E_INVALID_GRAPH"),
                       (-3, "BFS_E_ROOT_RANGE"), (-4, "BFS_E_NO_MEMORY"), (-5, "BFS_E_DEVICE"),
                       (-6, "BFS_E_UNKNOWN_TICKET"), (-7, "BFS_E_BUSY"), (-8, "BFS_E_SHUTDOWN"),
                       (-9, "BFS_E_INTERNAL")]:
        assert bfs.bfs_status_str(code) == name
    assert bfs.bfs_status_str(12345) == "BFS_E_UNKNOWN_STATUS"


def _load(off, col, flags=0):
    lib = bfs.load_library()
    h = ctypes.c_void_p()
    off = np.ascontiguousarray(off)
    col = np.ascontiguousarray(col, dtype=np.int32)
    rc = lib.bfs_graph_load_csr(len(off) - 1, len(col), off.ctypes.data, col.ctypes.data, flags, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("off,col,why", [
    (np.array([1, 2], dtype=np.int64), np.array([0], dtype=np.int32), "offsets[0] != 0"),
    (np.array([0, 2, 1], dtype=np.int64), np.array([0, 1], dtype=np.int32), "decreasing"),
    (np.array([0, 1, 1], dtype=np.int64), np.array([0, 1], dtype=np.int32), "offsets[n] != nnz"),
    (np.array([0, 1, 2], dtype=np.int64), np.array([0, 2], dtype=np.int32), "column >= n"),
    (np.array([0, 1, 2], dtype=np.int64), np.array([0, -1], dtype=np.int32), "negative column"),
    (np.array([0, 1, 2], dtype=np.int32), np.array([5, 0], dtype=np.int32), "column >= n, int32 offsets"),
])
def test_load_rejects_malformed_csr(off, col, why):
    flags = bfs.BFS_LOAD_OFFSETS_I32 if off.dtype == np.int32 else 0
    rc, h = _load(off, col, flags)
    assert rc == bfs.BFS_E_INVALID_GRAPH, why
    assert not h.value


def test_load_rejects_bad_sizes_and_nulls():
    lib = bfs.load_library()
    h = ctypes.c_void_p()
    off = np.zeros(2, dtype=np.int64)
    assert lib.bfs_graph_load_csr(0, 0, off.ctypes.data, None, 0, ctypes.byref(h)) == bfs.BFS_E_INVALID_GRAPH
    assert lib.bfs_graph_load_csr(1 << 31, 0, off.ctypes.data, None, 0, ctypes.byref(h)) == bfs.BFS_E_INVALID_GRAPH
    assert lib.bfs_graph_load_csr(1, -1, off.ctypes.data, None, 0, ctypes.byref(h)) == bfs.BFS_E_INVALID_GRAPH
    assert lib.bfs_graph_load_csr(1, 0, None, None, 0, ctypes.byref(h)) == bfs.BFS_E_INVALID_ARG
    assert lib.bfs_graph_load_csr(1, 0, off.ctypes.data, None, 0, None) == bfs.BFS_E_INVALID_ARG
    assert lib.bfs_graph_load_csr(1, 0, off.ctypes.data, None, 0x100, ctypes.byref(h)) == bfs.BFS_E_INVALID_ARG


def test_null_handles_rejected():
    lib = bfs.load_library()
    lv = np.zeros(4, dtype=np.int32)
    assert lib.bfs_run(None, 0, lv.ctypes.data, lv.ctypes.data, None, 0, None) == bfs.BFS_E_INVALID_ARG
    assert lib.bfs_run_batch(None, lv.ctypes.data, 1, lv.ctypes.data, lv.ctypes.data, None, 0, None) == \
        bfs.BFS_E_INVALID_ARG
    assert lib.bfs_graph_info(None, None, None, None) == bfs.BFS_E_INVALID_ARG
    assert lib.bfs_graph_free(None) == bfs.BFS_OK
    assert lib.bfs_autotune(None, lv.ctypes.data, 1, 0, None) == bfs.BFS_E_INVALID_ARG
    assert lib.bfs_server_submit(None, 0, 0, None) == bfs.BFS_E_INVALID_ARG
    assert lib.bfs_server_poll(None, 0, None, None, None) == bfs.BFS_E_INVALID_ARG
    assert lib.bfs_server_destroy(None) == bfs.BFS_OK


def test_server_refuses_single_root_workers():
    """The single-root worker route is closed (its fault is not explained): the
    request is refused before any device call."""
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_server_create(single_workers=2)
    assert e.value.status == bfs.BFS_E_INVALID_ARG


def test_python_binding_raises_with_status():
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_graph_load_csr(np.array([0, 1], dtype=np.int64), np.array([3], dtype=np.int32))
    assert e.value.status == bfs.BFS_E_INVALID_GRAPH
