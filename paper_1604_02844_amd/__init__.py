"""MI355X-native level-synchronous top-down BFS: Python binding of libbfs.so.

The functions below carry the names of the C ABI in ``include/bfs.h`` and only
marshal arguments: every step of the BFS runs in the HIP kernels of
``libbfs.so``. There is no CPU fallback — if the library is missing the calls
raise.

Buffers: device buffers are torch CUDA tensors (``data_ptr()``); host buffers
are numpy arrays. Streams are torch CUDA streams (``cuda_stream``) or None for
the current torch stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Any

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfs.so")

BFS_OK = 0
BFS_PENDING = 1
BFS_E_INVALID_ARG = -1
BFS_E_INVALID_GRAPH = -2
BFS_E_ROOT_RANGE = -3
BFS_E_NO_MEMORY = -4
BFS_E_DEVICE = -5
BFS_E_UNKNOWN_TICKET = -6
BFS_E_BUSY = -7
BFS_E_SHUTDOWN = -8
BFS_E_INTERNAL = -9

BFS_LOAD_DEVICE_PTRS = 0x1
BFS_LOAD_SKIP_VALIDATE = 0x2
BFS_LOAD_OFFSETS_I32 = 0x4
BFS_LOAD_SYMMETRIC = 0x8
BFS_OUT_HOST = 0x1
BFS_ASYNC = 0x2
BFS_HYBRID = 0x4
BFS_DETERMINISTIC = 0x10
BFS_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024

ABI_SYMBOLS = [
    "bfs_graph_load_csr", "bfs_graph_free", "bfs_graph_info", "bfs_graph_get_tunables",
    "bfs_graph_set_tunables", "bfs_run", "bfs_run_noalloc", "bfs_run_batch", "bfs_autotune", "bfs_server_create",
    "bfs_server_add_graph", "bfs_server_submit", "bfs_server_poll", "bfs_server_destroy",
    "bfs_status_str",
]


class BfsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {status_name(status)} ({status}){': ' + detail if detail else ''}")


class RunStats(ctypes.Structure):
    _fields_ = [("num_levels", ctypes.c_int32), ("num_roots", ctypes.c_int32), ("reached", ctypes.c_int64),
                ("arcs_scanned", ctypes.c_int64), ("edges_traversed", ctypes.c_int64),
                ("device_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tunables(ctypes.Structure):
    _fields_ = [("small_max_degree", ctypes.c_int32), ("wave_max_degree", ctypes.c_int32),
                ("chunk_arcs", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("batch_width", ctypes.c_int32),
                ("update_mode", ctypes.c_int32), ("hot_vertices", ctypes.c_int32),
                ("lds_visited", ctypes.c_int32), ("sparse_frontier", ctypes.c_int32),
                ("block_vertices", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("hub_bins", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerConfig(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("num_streams", ctypes.c_int32), ("max_instances_per_graph", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("single_workers", ctypes.c_int32), ("batch_min_queue", ctypes.c_int32)]


class RequestStats(ctypes.Structure):
    _fields_ = [("num_levels", ctypes.c_int32), ("graph_id", ctypes.c_int32), ("reached", ctypes.c_int64),
                ("arcs_scanned", ctypes.c_int64), ("edges_traversed", ctypes.c_int64),
                ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double), ("batched", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


_lib = None


def library_path() -> str:
    return LIB_PATH


def load_library():
    """Load libbfs.so (built by ``python -m paper_1604_02844_amd.build``); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libbfs.so not found at {LIB_PATH}; build it with "
                           "`python -m paper_1604_02844_amd.build` (no CPU fallback exists)")
    # PyTorch ships its own HIP runtime. Import it first, when it is installed,
    # so that libbfs.so binds to that same runtime: with the system runtime
    # loaded first, torch later finds no GPU in this process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    P = ctypes.POINTER
    sig = {
        "bfs_graph_load_csr": [i64, i64, vp, vp, u32, P(vp)],
        "bfs_graph_free": [vp],
        "bfs_graph_info": [vp, P(i64), P(i64), P(i64)],
        "bfs_graph_get_tunables": [vp, P(Tunables)],
        "bfs_graph_set_tunables": [vp, P(Tunables)],
        "bfs_run": [vp, i32, vp, vp, vp, u32, P(RunStats)],
        "bfs_run_noalloc": [vp, i32, vp, vp, vp, u32],
        "bfs_run_batch": [vp, vp, i32, vp, vp, vp, u32, P(RunStats)],
        "bfs_autotune": [vp, vp, i32, i32, P(Tunables)],
        "bfs_server_create": [P(ServerConfig), P(vp)],
        "bfs_server_add_graph": [vp, vp, P(i32)],
        "bfs_server_submit": [vp, i32, i32, P(u64)],
        "bfs_server_poll": [vp, u64, vp, vp, P(RequestStats)],
        "bfs_server_destroy": [vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.bfs_status_str.argtypes = [ctypes.c_int]
    lib.bfs_status_str.restype = ctypes.c_char_p
    lib.bfs_last_error.argtypes = []
    lib.bfs_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_name(status: int) -> str:
    try:
        return load_library().bfs_status_str(status).decode()
    except Exception:
        return str(status)


def bfs_status_str(status: int) -> str:
    return load_library().bfs_status_str(status).decode()


def _check(rc: int, where: str) -> int:
    if rc < 0:
        detail = load_library().bfs_last_error().decode(errors="replace")
        raise BfsError(rc, where, detail)
    return rc


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x) -> int:
    if x is None:
        return 0
    if _is_torch(x):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return x.ctypes.data
    raise TypeError(f"unsupported buffer type {type(x)}")


def _stream_ptr(stream) -> int:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class Graph:
    """A resident graph (owns the ``bfs_graph*`` handle)."""

    def __init__(self, handle: int, n: int, nnz: int, keepalive: Any = None):
        self.handle = handle
        self.n = n
        self.nnz = nnz
        self._keepalive = keepalive

    def __del__(self):
        try:
            if self.handle:
                bfs_graph_free(self)
        except Exception:
            pass


def bfs_graph_load_csr(offsets, cols, flags: int = 0) -> Graph:
    """Upload (host numpy) or borrow (torch CUDA tensors) a CSR graph.

    int32 offsets set BFS_LOAD_OFFSETS_I32; torch CUDA tensors set
    BFS_LOAD_DEVICE_PTRS and are kept alive by the returned Graph.
    """
    lib = load_library()
    keep = None
    if _is_torch(offsets):
        import torch

        if offsets.dtype == torch.int32:
            flags |= BFS_LOAD_OFFSETS_I32
        elif offsets.dtype != torch.int64:
            raise TypeError("offsets must be int32 or int64")
        if cols.dtype != torch.int32:
            raise TypeError("cols must be int32")
        if offsets.is_cuda:
            flags |= BFS_LOAD_DEVICE_PTRS
            keep = (offsets, cols)
        n = offsets.numel() - 1
        nnz = cols.numel()
    else:
        offsets = np.ascontiguousarray(offsets)
        if offsets.dtype == np.int32:
            flags |= BFS_LOAD_OFFSETS_I32
        elif offsets.dtype != np.int64:
            offsets = offsets.astype(np.int64)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        n = len(offsets) - 1
        nnz = len(cols)
    h = ctypes.c_void_p()
    _check(lib.bfs_graph_load_csr(n, nnz, _ptr(offsets), _ptr(cols), flags, ctypes.byref(h)),
           "bfs_graph_load_csr")
    return Graph(h.value, n, nnz, keep)


def bfs_graph_free(g: Graph) -> None:
    if g.handle:
        _check(load_library().bfs_graph_free(g.handle), "bfs_graph_free")
        g.handle = 0
        g._keepalive = None


def bfs_graph_info(g: Graph) -> dict:
    n, nnz, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load_library().bfs_graph_info(g.handle, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(b)),
           "bfs_graph_info")
    return {"n": n.value, "nnz": nnz.value, "device_bytes": b.value}


def bfs_graph_get_tunables(g: Graph) -> dict:
    t = Tunables()
    _check(load_library().bfs_graph_get_tunables(g.handle, ctypes.byref(t)), "bfs_graph_get_tunables")
    return t.as_dict()


def bfs_graph_set_tunables(g: Graph, **kw) -> dict:
    t = Tunables()
    for k, v in kw.items():
        setattr(t, k, int(v))
    _check(load_library().bfs_graph_set_tunables(g.handle, ctypes.byref(t)), "bfs_graph_set_tunables")
    return bfs_graph_get_tunables(g)


def bfs_run(g: Graph, root: int, levels, parents, stream=None, flags: int = 0, stats: bool = True):
    """One BFS. levels/parents: int32 torch CUDA tensors (device) or numpy arrays (host)."""
    host = isinstance(levels, np.ndarray)
    if host:
        flags |= BFS_OUT_HOST
    st = RunStats() if stats and not (flags & BFS_ASYNC) else None
    rc = load_library().bfs_run(g.handle, int(root), _ptr(levels), _ptr(parents),
                                0 if host and stream is None else _stream_ptr(stream), flags,
                                ctypes.byref(st) if st is not None else None)
    _check(rc, "bfs_run")
    return st.as_dict() if st is not None else None


def bfs_run_noalloc(g: Graph, root: int, levels, parents, stream=None, flags: int = 0) -> None:
    """One BFS with every scratch buffer in the library's static device array.
    levels/parents: int32 torch CUDA tensors. Returns when the run is done."""
    rc = load_library().bfs_run_noalloc(g.handle, int(root), _ptr(levels), _ptr(parents), _stream_ptr(stream),
                                        flags)
    _check(rc, "bfs_run_noalloc")


def bfs_run_batch(g: Graph, roots, levels, parents, stream=None, flags: int = 0, stats: bool = True):
    """Multi-source BFS; levels/parents are [num_roots, n] int32 (row-major)."""
    roots = np.ascontiguousarray(roots, dtype=np.int32)
    host = isinstance(levels, np.ndarray)
    if host:
        flags |= BFS_OUT_HOST
    st = RunStats() if stats and not (flags & BFS_ASYNC) else None
    rc = load_library().bfs_run_batch(g.handle, roots.ctypes.data, len(roots), _ptr(levels), _ptr(parents),
                                      0 if host and stream is None else _stream_ptr(stream), flags,
                                      ctypes.byref(st) if st is not None else None)
    _check(rc, "bfs_run_batch")
    return st.as_dict() if st is not None else None


def bfs_autotune(g: Graph, roots, mode: int = 0) -> dict:
    roots = np.ascontiguousarray(roots, dtype=np.int32)
    t = Tunables()
    _check(load_library().bfs_autotune(g.handle, roots.ctypes.data, len(roots), mode, ctypes.byref(t)),
           "bfs_autotune")
    return t.as_dict()


class Server:
    def __init__(self, handle: int):
        self.handle = handle
        self.graphs: list[Graph] = []

    def __del__(self):
        try:
            if self.handle:
                bfs_server_destroy(self)
        except Exception:
            pass


def bfs_server_create(mem_budget_bytes: int = 0, max_slots: int = 0, num_streams: int = 0,
                      max_instances_per_graph: int = 0, single_workers: int = 0, batch_min_queue: int = 0) -> Server:
    cfg = ServerConfig(mem_budget_bytes, max_slots, num_streams, max_instances_per_graph, 0, single_workers,
                       batch_min_queue)
    h = ctypes.c_void_p()
    _check(load_library().bfs_server_create(ctypes.byref(cfg), ctypes.byref(h)), "bfs_server_create")
    return Server(h.value)


def bfs_server_add_graph(s: Server, g: Graph) -> int:
    gid = ctypes.c_int32()
    _check(load_library().bfs_server_add_graph(s.handle, g.handle, ctypes.byref(gid)), "bfs_server_add_graph")
    s.graphs.append(g)
    return gid.value


def bfs_server_submit(s: Server, graph_id: int, root: int) -> int:
    t = ctypes.c_uint64()
    _check(load_library().bfs_server_submit(s.handle, graph_id, int(root), ctypes.byref(t)), "bfs_server_submit")
    return t.value


def bfs_server_poll(s: Server, ticket: int, levels=None, parents=None):
    """Return None while pending, else the request's stats dict (results copied out)."""
    st = RequestStats()
    rc = load_library().bfs_server_poll(s.handle, ticket, _ptr(levels), _ptr(parents), ctypes.byref(st))
    _check(rc, "bfs_server_poll")
    return None if rc == BFS_PENDING else st.as_dict()


def bfs_server_destroy(s: Server) -> None:
    if s.handle:
        _check(load_library().bfs_server_destroy(s.handle), "bfs_server_destroy")
        s.handle = 0
