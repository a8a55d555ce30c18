#!/usr/bin/env python3
"""Benchmark of the BFS hot path on one MI355X.

Default workload: single-root top-down BFS on an R-MAT graph of scale 20
(1,048,576 vertices), edgefactor 16, initiator .57/.19/.19/.05, ids permuted,
symmetrised and deduplicated, int32 columns with int64 offsets, 64 seeded roots
of degree > 0. One step = one BFS from each of the 64 roots.

Printed: one JSON line with the harmonic mean of per-root GTEPS (m = arcs/2 of
the root's component, t = device time of the run from HIP events on the run's
stream), the roofline object of the BFS kernel (algorithmic bytes per launch /
average launch duration vs 8 TB/s HBM) and the CPU oracle's rate on a bounded
sample of the same roots.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(n: int, reached: int, arcs: int, levels: int, off_bytes: int) -> int:
    """Compulsory traffic of one BFS: init 8n, level+parent writes 8R, two
    offsets per expanded vertex, one 4-byte column per scanned arc, and per
    level a read of the frontier bitmap, a read of the visited footprint and a
    clear+write of the next bitmap (3 * n/8)."""
    return 8 * n + 8 * reached + 2 * off_bytes * reached + 4 * arcs + levels * 3 * (n // 8)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=20)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--root-seed", type=int, default=2)
    ap.add_argument("--offsets-i32", action="store_true", help="keep 4-byte offsets on the device")
    ap.add_argument("--cpu-sample-roots", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true", help="run the autotuner on 4 roots first")
    ap.add_argument("--tunables", default="", help='JSON object of bfs_tunables fields, e.g. {"update_mode": 2}')
    ap.add_argument("--details", default="", help="write per-root records (JSON) to this path")
    return ap.parse_args()


def main() -> int:
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the batched and serving patterns shard by replicating graphs per GPU; see DESIGN.md)",
              file=sys.stderr)
        return 2

    import torch

    import graphgen
    import paper_1604_02844_amd as bfs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    bfs.load_library()

    t_gen = time.perf_counter()
    g = graphgen.cached("rmat", scale=args.scale, edgefactor=args.edgefactor, seed=args.seed)
    roots = graphgen.pick_roots(g, args.roots, seed=args.root_seed)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] graph {g.name}: n={g.n} nnz={g.nnz} ({t_gen:.1f}s), {len(roots)} roots", file=sys.stderr,
          flush=True)
    dg = bfs.bfs_graph_load_csr(g.offsets_i32() if args.offsets_i32 else g.offsets, g.cols)
    if args.tunables:
        bfs.bfs_graph_set_tunables(dg, **json.loads(args.tunables))
    if args.tune:
        best = bfs.bfs_autotune(dg, roots[:4], 0)
        print(f"[bench] tuned: {best}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    lv = torch.empty(g.n, dtype=torch.int32, device=dev)
    pa = torch.empty(g.n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        recs = []
        for r in roots:
            st = bfs.bfs_run(dg, int(r), lv, pa, stream=stream)
            recs.append((int(r), st))
        return recs

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_recs = []
    for i in range(args.steps):
        all_recs += step()
        print(f"[bench] step {i + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    off_bytes = 4 if args.offsets_i32 else 8
    inv_teps = 0.0
    bytes_total = 0
    ms_total = 0.0
    per_root = []
    for r, st in all_recs:
        t = st["device_ms"] * 1e-3
        m = st["edges_traversed"]
        inv_teps += t / m if m > 0 else float("inf")
        b = algorithmic_bytes(g.n, st["reached"], st["arcs_scanned"], st["num_levels"], off_bytes)
        bytes_total += b
        ms_total += st["device_ms"]
        per_root.append({"root": r, "ms": st["device_ms"], "m": m, "reached": st["reached"],
                         "arcs": st["arcs_scanned"], "levels": st["num_levels"], "bytes_alg": b,
                         "gteps": m / t / 1e9 if t > 0 else None})
    hm_gteps = len(all_recs) / inv_teps / 1e9 if inv_teps > 0 else 0.0
    launches = len(all_recs)
    avg_ms = ms_total / launches
    achieved = (bytes_total / launches) / (avg_ms * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        sample = roots[: args.cpu_sample_roots]
        threads = min(len(sample), os.cpu_count() or 1, 16)
        res, cwall, used = oracle.bfs_many(g.offsets, g.cols, sample, threads=threads)
        inv = sum(t / s["edges"] for _, t, s in res if s["edges"] > 0)
        cpu = {"value": round(len(res) / inv / 1e9, 4) if inv > 0 else 0.0, "unit": "GTEPS (harmonic mean over roots)",
               "cores": used, "kind": "oracle",
               "sample": f"{len(sample)} of the {len(roots)} roots, one serial queue BFS per host thread, "
                         f"{used} threads, {cwall:.2f}s wall; per-root time on one core",
               "throughput_gteps": round(sum(s["edges"] for _, _, s in res) / cwall / 1e9, 4)}

    out = {
        "metric": "GTEPS (harmonic mean over roots) + % HBM roofline",
        "value": round(hm_gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"single-root top-down BFS, R-MAT scale {args.scale}, edgefactor {args.edgefactor}, "
                               f"A/B/C/D=.57/.19/.19/.05, permuted, symmetrised, deduplicated, int32 cols, "
                               f"int{off_bytes * 8} offsets, {len(roots)} seeded roots of degree>0",
                   "n": g.n, "nnz": g.nnz, "roots": len(roots), "step": f"{len(roots)} BFS runs",
                   "tunables": bfs.bfs_graph_get_tunables(dg)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_bfs_single", "avg_launch_ms": round(avg_ms, 4),
                     "bytes_alg_per_launch": int(bytes_total / launches)},
        "cpu_baseline": cpu,
    }
    if args.details:
        with open(args.details, "w") as f:
            json.dump({"per_root": per_root, "summary": out}, f, indent=1)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
