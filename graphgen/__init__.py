"""Seeded synthetic input graphs shared by the GPU library's tests/bench and the oracle.

This module only *generates inputs*: R-MAT/Kronecker and Erdos-Renyi graphs
(host C in ``gen.c``), closed-form families (path, cycle, star, complete graph,
2-D grid, heap-numbered binary tree) and seeded root samples. It holds none of
the BFS arithmetic and imports neither the oracle nor the GPU package.

The R-MAT parameters follow the paper's workload (section "Input graph"):
2^SCALE vertices, edgefactor * 2^SCALE drawn edges, initiator A=.57, B=.19,
C=.19, D=.05; edges are bidirectional. Readings where the paper is silent
(no initiator noise, seeded Fisher-Yates relabelling, SplitMix64 counter-based
draws, self-loop/duplicate removal) are stated in ``gen.c``.
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def build(force: bool = False) -> str:
    """Compile ``gen.c`` into ``libgraphgen.so`` (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, u64, i32p, i64p = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p
        lib.gg_rmat.restype = i64
        lib.gg_rmat.argtypes = [ctypes.c_int, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                u64, i64, ctypes.c_int, i64p, i32p]
        lib.gg_er.restype = i64
        lib.gg_er.argtypes = [i64, i64, u64, ctypes.c_int, i64p, i32p]
        lib.gg_rmat_edges.restype = ctypes.c_int
        lib.gg_rmat_edges.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      u64, i64, i64, i64p, i64p]
        lib.gg_pick_roots.restype = i64
        lib.gg_pick_roots.argtypes = [i64, i64p, i64, u64, i32p]
        lib.gg_permutation.restype = ctypes.c_int
        lib.gg_permutation.argtypes = [i64, u64, i32p]
        lib.gg_uniform_u64.restype = ctypes.c_int
        lib.gg_uniform_u64.argtypes = [u64, u64, i64, u64, ctypes.c_void_p]
        lib.gg_uniform_f64.restype = ctypes.c_int
        lib.gg_uniform_f64.argtypes = [u64, u64, i64, ctypes.c_void_p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


@dataclass
class Csr:
    """A CSR graph: row ``v`` is ``cols[offsets[v]:offsets[v+1]]`` (out-neighbours)."""

    n: int
    offsets: np.ndarray  # int64[n+1]
    cols: np.ndarray  # int32[nnz]
    name: str = "graph"

    @property
    def nnz(self) -> int:
        return int(self.offsets[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)

    def offsets_i32(self) -> np.ndarray:
        if self.nnz > np.iinfo(np.int32).max:
            raise ValueError("graph too large for int32 offsets")
        return self.offsets.astype(np.int32)


def rmat(scale: int, edgefactor: int = 16, A: float = RMAT_A, B: float = RMAT_B, C: float = RMAT_C,
         seed: int = 1, perm_seed: int | None = None, threads: int = 0) -> Csr:
    """Symmetric, deduplicated R-MAT graph with ids relabelled by a seeded permutation.

    ``perm_seed`` defaults to ``seed``; pass ``-1`` to keep the raw Kronecker ids.
    """
    lib = _load()
    n = 1 << scale
    m = edgefactor * n
    offsets = np.empty(n + 1, dtype=np.int64)
    cols = np.empty(2 * m, dtype=np.int32)
    ps = seed if perm_seed is None else perm_seed
    nnz = lib.gg_rmat(scale, edgefactor, A, B, C, seed, ps, threads, _ptr(offsets), _ptr(cols))
    if nnz < 0:
        raise RuntimeError(f"gg_rmat failed ({nnz})")
    return Csr(n, offsets, cols[:nnz], name=f"rmat{scale}_ef{edgefactor}_s{seed}")


def er(n: int, avg_degree: float, seed: int = 1, threads: int = 0) -> Csr:
    """Erdos-Renyi graph: M = n*avg_degree/2 uniform pairs, symmetrised and deduplicated."""
    lib = _load()
    m = int(round(n * avg_degree / 2))
    offsets = np.empty(n + 1, dtype=np.int64)
    cols = np.empty(max(2 * m, 1), dtype=np.int32)
    nnz = lib.gg_er(n, m, seed, threads, _ptr(offsets), _ptr(cols))
    if nnz < 0:
        raise RuntimeError(f"gg_er failed ({nnz})")
    return Csr(n, offsets, cols[:nnz], name=f"er{n}_d{avg_degree:g}_s{seed}")


def rmat_edges(scale: int, count: int, seed: int = 1, e0: int = 0,
               A: float = RMAT_A, B: float = RMAT_B, C: float = RMAT_C):
    """Raw R-MAT draws (before relabelling, symmetrisation and deduplication)."""
    lib = _load()
    src = np.empty(count, dtype=np.int64)
    dst = np.empty(count, dtype=np.int64)
    if lib.gg_rmat_edges(scale, A, B, C, seed, e0, count, _ptr(src), _ptr(dst)) != 0:
        raise RuntimeError("gg_rmat_edges failed")
    return src, dst


def permutation(n: int, seed: int) -> np.ndarray:
    lib = _load()
    p = np.empty(n, dtype=np.int32)
    lib.gg_permutation(n, seed, _ptr(p))
    return p


def pick_roots(g: Csr, k: int, seed: int = 2) -> np.ndarray:
    """``k`` distinct roots of degree > 0 in a fixed seeded order."""
    lib = _load()
    out = np.empty(max(k, 1), dtype=np.int32)
    got = lib.gg_pick_roots(g.n, _ptr(g.offsets), k, seed, _ptr(out))
    if got < 0:
        raise RuntimeError("gg_pick_roots failed")
    return out[:got].copy()


def uniform_u64(seed: int, stream: int, count: int, bound: int = 0) -> np.ndarray:
    lib = _load()
    out = np.empty(count, dtype=np.uint64)
    lib.gg_uniform_u64(seed, stream, count, bound, out.ctypes.data)
    return out


def uniform_f64(seed: int, stream: int, count: int) -> np.ndarray:
    lib = _load()
    out = np.empty(count, dtype=np.float64)
    lib.gg_uniform_f64(seed, stream, count, out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# Closed-form families and small hand-made graphs (numpy, tiny to medium n)
# ---------------------------------------------------------------------------

def from_edges(n: int, src, dst, symmetric: bool = True, dedupe: bool = True,
               drop_self_loops: bool = True, sort_rows: bool = True, name: str = "edges") -> Csr:
    """CSR from an arc list. With ``symmetric`` every pair gives both directions."""
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("endpoint out of range")
    if symmetric:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    if drop_self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    if dedupe:
        key = np.unique(src * n + dst)
        src, dst = key // n, key % n
    elif sort_rows:
        order = np.lexsort((dst, src))
        src, dst = src[order], dst[order]
    else:
        order = np.argsort(src, kind="stable")
        src, dst = src[order], dst[order]
    counts = np.bincount(src, minlength=n) if src.size else np.zeros(n, dtype=np.int64)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return Csr(n, offsets, dst.astype(np.int32), name=name)


def path(n: int) -> Csr:
    v = np.arange(n - 1)
    return from_edges(n, v, v + 1, name=f"path{n}")


def cycle(n: int) -> Csr:
    v = np.arange(n)
    return from_edges(n, v, (v + 1) % n, name=f"cycle{n}")


def star(n: int) -> Csr:
    """Centre 0 joined to leaves 1..n-1."""
    v = np.arange(1, n)
    return from_edges(n, np.zeros_like(v), v, name=f"star{n}")


def complete(n: int) -> Csr:
    a, b = np.triu_indices(n, 1)
    return from_edges(n, a, b, name=f"complete{n}")


def grid(rows: int, cols_: int) -> Csr:
    """4-neighbour grid, vertex id = row * cols + col."""
    idx = np.arange(rows * cols_).reshape(rows, cols_)
    a = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    b = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return from_edges(rows * cols_, a, b, name=f"grid{rows}x{cols_}")


def binary_tree(n: int) -> Csr:
    """Complete binary tree in heap numbering: parent of v is (v-1)//2."""
    v = np.arange(1, n)
    return from_edges(n, (v - 1) // 2, v, name=f"bintree{n}")


def disjoint(g1: Csr, g2: Csr) -> Csr:
    """Disjoint union; g2's ids are shifted by g1.n."""
    offsets = np.concatenate([g1.offsets, g2.offsets[1:] + g1.nnz])
    cols = np.concatenate([g1.cols, g2.cols + g1.n]).astype(np.int32)
    return Csr(g1.n + g2.n, offsets, cols, name=f"{g1.name}+{g2.name}")


def empty(n: int) -> Csr:
    return Csr(n, np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32), name=f"empty{n}")


# ---------------------------------------------------------------------------
# Optional on-disk cache for large generated graphs
# ---------------------------------------------------------------------------

def cache_dir() -> str:
    d = os.environ.get("BFS_GRAPH_CACHE", "/tmp/bfs_graph_cache")
    os.makedirs(d, exist_ok=True)
    return d


def cached(kind: str, **params) -> Csr:
    """Generate (or load from the cache) ``rmat``/``er`` graphs by parameters."""
    key = kind + "_" + "_".join(f"{k}{params[k]}" for k in sorted(params))
    h = hashlib.sha1(key.encode()).hexdigest()[:12]
    base = os.path.join(cache_dir(), f"{kind}_{h}")
    if os.path.exists(base + ".done"):
        off = np.load(base + "_off.npy", mmap_mode="r")
        col = np.load(base + "_col.npy", mmap_mode="r")
        return Csr(len(off) - 1, np.asarray(off), np.asarray(col), name=key)
    g = rmat(**params) if kind == "rmat" else er(**params)
    try:
        np.save(base + "_off.npy", g.offsets)
        np.save(base + "_col.npy", g.cols)
        open(base + ".done", "w").close()
    except OSError:
        pass
    g.name = key
    return g
