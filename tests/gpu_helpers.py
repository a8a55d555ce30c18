"""Shared helpers for the GPU parity tests: run the HIP path through the C ABI,
run the oracle on the same seeded input, compare levels exactly and validate
parents (V1-V4)."""
from __future__ import annotations

import numpy as np

import oracle
import paper_1604_02844_amd as bfs


def torch_mod():
    import torch

    return torch


def load(g, offsets_i32: bool = False, device_ptrs: bool = False, symmetric: bool = False):
    off = g.offsets_i32() if offsets_i32 else g.offsets
    flags = bfs.BFS_LOAD_SYMMETRIC if symmetric else 0
    if device_ptrs:
        torch = torch_mod()
        return bfs.bfs_graph_load_csr(torch.from_numpy(off).cuda(), torch.from_numpy(g.cols).cuda(), flags)
    return bfs.bfs_graph_load_csr(off, g.cols, flags)


def gpu_run(dg, root: int, flags: int = 0):
    torch = torch_mod()
    lv = torch.empty(dg.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(dg.n, dtype=torch.int32, device="cuda")
    st = bfs.bfs_run(dg, int(root), lv, pa, flags=flags)
    return lv.cpu().numpy(), pa.cpu().numpy(), st


def check_root(g, dg, root: int, rows_sorted: bool = True, expected_levels=None, flags: int = 0):
    print(f"[case] bfs_run {g.name} n={g.n} nnz={g.nnz} root={root} flags={flags}", flush=True)
    lv, pa, st = gpu_run(dg, root, flags)
    ref, _, ost = oracle.bfs(g.offsets, g.cols, int(root))
    if expected_levels is not None:
        assert np.array_equal(ref, expected_levels), "oracle disagrees with the closed form"
    code, bad = oracle.validate(g.offsets, g.cols, int(root), ref, lv, pa, rows_sorted=rows_sorted)
    assert code == 0, (f"{g.name} root {root}: {oracle.CHECK_NAMES[code]} at vertex {bad} "
                       f"(gpu level {lv[bad] if bad >= 0 else None}, oracle {ref[bad] if bad >= 0 else None})")
    assert st["reached"] == ost["reached"], (st, ost)
    assert st["arcs_scanned"] == ost["arcs"], (st, ost)
    assert st["num_levels"] == ost["levels"], (st, ost)
    return lv, pa, st
