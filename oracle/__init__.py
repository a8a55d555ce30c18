"""CPU oracle for top-down BFS — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It wraps ``bfs_oracle.c`` (plain C, built
with gcc) and shares no code with the GPU library.

* ``bfs``       serial FIFO-queue BFS in the form of the paper's serial top-down
                algorithm (section 3.1, Algorithm 1); unique ``levels`` plus the
                FIFO-first ``parents``.
* ``validate``  V1-V4 check of a candidate ``(levels, parents)`` against the
                oracle's levels (the parent choice is free; section 3.2).
* ``certify``   V2-V5 check of a candidate on its own (no oracle levels): exact
                when levels are hop distances and parents form a BFS tree.
* ``bfs_many``  the same serial BFS from several roots, one root per host
                thread, used only to time the CPU baseline.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CHECK_NAMES = {0: "ok", 1: "V1 levels differ", 2: "V2 root", 3: "V3 reached set / parent -1",
               4: "V4 parent not adjacent one level up", 5: "V5 arc skips a level or leaves the reached set"}


def build(force: bool = False, src: str = _SRC, out: str = _LIB_PATH) -> str:
    """Compile the oracle with gcc (no HIP headers, no GPU library)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, out)
    return out


def load_library(path: str):
    lib = ctypes.CDLL(path)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.oracle_bfs.restype = ctypes.c_int
    lib.oracle_bfs.argtypes = [i64, vp, vp, i64, vp, vp, vp]
    lib.oracle_validate.restype = ctypes.c_int
    lib.oracle_validate.argtypes = [i64, vp, vp, i64, vp, vp, vp, ctypes.c_int, vp]
    lib.oracle_certify.restype = ctypes.c_int
    lib.oracle_certify.argtypes = [i64, vp, vp, i64, vp, vp, ctypes.c_int, vp]
    lib.oracle_min_parents.restype = ctypes.c_int
    lib.oracle_min_parents.argtypes = [i64, vp, vp, i64, vp, vp, vp]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = load_library(_LIB_PATH)
    return _lib


def _as64(offsets) -> np.ndarray:
    return np.ascontiguousarray(offsets, dtype=np.int64)


def _as32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def bfs(offsets, cols, root: int, lib=None):
    """Return ``(levels, parents, stats)``; stats has R, A, L and m = A/2."""
    lib = lib or _load()
    off = _as64(offsets)
    col = _as32(cols)
    n = len(off) - 1
    levels = np.empty(n, dtype=np.int32)
    parents = np.empty(n, dtype=np.int32)
    st = np.zeros(3, dtype=np.int64)
    rc = lib.oracle_bfs(n, off.ctypes.data, col.ctypes.data, int(root), levels.ctypes.data,
                        parents.ctypes.data, st.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_bfs failed ({rc})")
    return levels, parents, {"reached": int(st[0]), "arcs": int(st[1]), "levels": int(st[2]),
                             "edges": int(st[1]) // 2}


def validate(offsets, cols, root: int, ref_levels, levels, parents, rows_sorted: bool = True,
             lib=None):
    """Return ``(code, bad_vertex)``; code 0 means V1-V4 all hold."""
    lib = lib or _load()
    off = _as64(offsets)
    col = _as32(cols)
    n = len(off) - 1
    rl, lv, pa = _as32(ref_levels), _as32(levels), _as32(parents)
    if not (len(rl) == len(lv) == len(pa) == n):
        raise ValueError("length mismatch")
    bad = np.full(1, -1, dtype=np.int64)
    rc = lib.oracle_validate(n, off.ctypes.data, col.ctypes.data, int(root), rl.ctypes.data,
                             lv.ctypes.data, pa.ctypes.data, int(bool(rows_sorted)), bad.ctypes.data)
    if rc < 0:
        raise ValueError(f"oracle_validate argument error ({rc})")
    return rc, int(bad[0])


def certify(offsets, cols, root: int, levels, parents, rows_sorted: bool = True, lib=None):
    """V2-V5 without oracle levels: ``(code, bad_vertex)``, code 0 = levels are the
    hop distances and parents a BFS tree."""
    lib = lib or _load()
    off = _as64(offsets)
    col = _as32(cols)
    n = len(off) - 1
    lv, pa = _as32(levels), _as32(parents)
    if not (len(lv) == len(pa) == n):
        raise ValueError("length mismatch")
    bad = np.full(1, -1, dtype=np.int64)
    rc = lib.oracle_certify(n, off.ctypes.data, col.ctypes.data, int(root), lv.ctypes.data, pa.ctypes.data,
                            int(bool(rows_sorted)), bad.ctypes.data)
    if rc < 0:
        raise ValueError(f"oracle_certify argument error ({rc})")
    return rc, int(bad[0])


def min_parents(offsets, cols, root: int, levels, lib=None):
    """Deterministic predecessors from a level array: the least in-neighbour one
    level up of every reached non-root vertex (root: itself; unreached: -1)."""
    lib = lib or _load()
    off = _as64(offsets)
    col = _as32(cols)
    n = len(off) - 1
    lv = _as32(levels)
    if len(lv) != n:
        raise ValueError("length mismatch")
    pa = np.empty(n, dtype=np.int32)
    bad = np.full(1, -1, dtype=np.int64)
    rc = lib.oracle_min_parents(n, off.ctypes.data, col.ctypes.data, int(root), lv.ctypes.data, pa.ctypes.data,
                                bad.ctypes.data)
    if rc != 0:
        raise ValueError(f"oracle_min_parents failed ({rc}, vertex {int(bad[0])})")
    return pa


def bfs_many(offsets, cols, roots, threads: int | None = None):
    """Serial BFS from each root, roots spread over ``threads`` host threads.

    Returns ``(per_root, wall_s, threads)`` where per_root is a list of
    ``(root, seconds, stats)``; each root's time covers initialisation through
    the end of its queue loop.
    """
    lib = _load()
    off = _as64(offsets)
    col = _as32(cols)
    n = len(off) - 1
    threads = threads or os.cpu_count() or 1

    def one(r):
        levels = np.empty(n, dtype=np.int32)
        parents = np.empty(n, dtype=np.int32)
        st = np.zeros(3, dtype=np.int64)
        t0 = time.perf_counter()
        rc = lib.oracle_bfs(n, off.ctypes.data, col.ctypes.data, int(r), levels.ctypes.data,
                            parents.ctypes.data, st.ctypes.data)
        t1 = time.perf_counter()
        if rc != 0:
            raise ValueError(f"oracle_bfs failed ({rc})")
        return int(r), t1 - t0, {"reached": int(st[0]), "arcs": int(st[1]), "levels": int(st[2]),
                                 "edges": int(st[1]) // 2}

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        res = list(ex.map(one, list(roots)))
    return res, time.perf_counter() - t0, threads
