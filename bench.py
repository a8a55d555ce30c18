#!/usr/bin/env python3
"""Benchmark of the BFS hot path on one MI355X.

Default (--mode single): single-root top-down BFS on an R-MAT graph of scale 24
(16,777,216 vertices), edgefactor 16, initiator .57/.19/.19/.05, ids permuted,
symmetrised and deduplicated, int32 columns with int64 offsets, 64 seeded roots
of degree > 0. One step = one BFS from each of the 64 roots. Printed: one JSON
line with the harmonic mean of per-root GTEPS (m = arcs/2 of the root's
component, t = device time of the run from HIP events on the run's stream), the
roofline object of the BFS (algorithmic bytes per run / average run duration vs
8 TB/s HBM), the CPU oracle's rate on a bounded sample of the same roots, and a
`batch` object: 64 roots of an R-MAT scale-22 graph in one multi-source run
against the same roots one at a time, with its own algorithmic bytes and
roofline fraction (--no-batch leaves it out).

--mode batch: multi-source BFS (R-MAT scale 22 with 64 roots; Erdos-Renyi 2^22,
average degree 16, with 8/32/64 roots), aggregate GTEPS against the same roots
run one at a time, each case with its algorithmic bytes and roofline fraction.
--mode serve: the continuous-batching server on 8 resident graphs, Poisson
arrivals, Zipf(1.1) graph choice; p50/p99 latency and aggregate GTEPS per rate,
against the same trace replayed through single-root runs in FIFO order.
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


def hybrid_algorithmic_bytes(lv, deg, off_bytes: int) -> int:
    """Compulsory traffic of one direction-optimising BFS, from its level array
    (torch int32 [n] on the device) and the degrees: init 8n, level+parent
    writes 8R, three bitmap passes per level (3 * n/8), and per level the
    cheaper of the two directions' compulsory reads: top-down, two offsets per
    frontier vertex and every arc of its row; bottom-up, two offsets per
    unvisited vertex with arcs, one arc for each one found at this level and
    every arc of each one that stays unvisited. A lower bound for any choice
    of directions."""
    n = lv.numel()
    L = int(lv.max().item()) + 1
    has = deg > 0
    total = 8 * n + 8 * int((lv >= 0).sum().item()) + L * 3 * (n // 8)
    for k in range(L):
        fr = lv == k
        td = 2 * off_bytes * int(fr.sum().item()) + 4 * int(deg[fr].sum().item())
        unv = ((lv > k) | (lv < 0)) & has
        disc = lv == k + 1
        bu = 2 * off_bytes * int(unv.sum().item()) + 4 * (int(disc.sum().item()) + int(deg[unv & ~disc].sum().item()))
        total += min(td, bu)
    return total


def batch_algorithmic_bytes(n: int, roots: int, levels: int, rows: int, row_arcs: int, discovered: int,
                            off_bytes: int) -> int:
    """Compulsory traffic of one multi-source run of `roots` roots: per level a
    sweep of the three 64-bit mask arrays (3 * 8n); per active row (a vertex
    holding any root's frontier bit, counted once per level) two offsets and its
    4-byte columns; the output rows of every root (8n each); and one level and
    one parent write per (root, vertex) discovery."""
    return levels * 24 * n + 2 * off_bytes * rows + 4 * row_arcs + roots * 8 * n + 8 * discovered


def batch_active_rows(lv, deg, levels: int):
    """From a batch's level rows (torch int32 [B, n] on the device; measurement
    only, after the timed run): per level, the vertices reached by any root at
    that level and the sum of their degrees. Returns (rows, row_arcs) summed
    over levels."""
    rows = arcs = 0
    for k in range(levels):
        act = (lv == k).any(0)
        rows += int(act.sum().item())
        arcs += int(deg[act].sum().item())
    return rows, arcs


def host_info() -> dict:
    """CPU model, logical CPUs, CPUs this process may use, RAM and the oracle's
    compiler, for the CPU baseline record."""
    import platform
    import subprocess

    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem_gib = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal:"):
                    mem_gib = round(int(line.split()[1]) / 2**20, 1)
                    break
    except OSError:
        pass
    try:
        cc = subprocess.run(["gcc", "--version"], capture_output=True, text=True).stdout.splitlines()[0]
    except (OSError, IndexError):
        cc = "gcc"
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "ram_gib": mem_gib, "compiler": f"{cc}; flags -O2 -fPIC -shared"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--edgefactor", type=int, default=16)
    ap.add_argument("--roots", type=int, default=64)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--root-seed", type=int, default=2)
    ap.add_argument("--offsets-i32", action="store_true", help="keep 4-byte offsets on the device")
    ap.add_argument("--hybrid", action="store_true",
                    help="direction-optimising runs (BFS_HYBRID): large levels bottom-up, not top-down")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="single-core seconds of oracle work in the CPU baseline")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="most host threads for the CPU baseline (the host CPU share of one GPU)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="leave the R-MAT 22 batched object out of the line")
    ap.add_argument("--tune", action="store_true", help="run the autotuner on 4 roots first")
    ap.add_argument("--no-shipped-tunables", action="store_true",
                    help="library defaults instead of the shipped autotuner result for this configuration")
    ap.add_argument("--tunables", default="", help='JSON object of bfs_tunables fields, e.g. {"update_mode": 2}')
    ap.add_argument("--details", default="", help="write per-root records (JSON) to this path")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="also run a plain copy kernel of BYTES (read and written) for counter scaling")
    ap.add_argument("--mode", default="single", choices=["single", "batch", "serve", "ceilings"])
    ap.add_argument("--batch-case", default="", metavar="GRAPH:ROOTS",
                    help="batch: only this case (rmat22 or er22_d16, with a root count), in the default launch "
                         "form only, e.g. rmat22:64 (for a kernel trace of one case)")
    ap.add_argument("--rates", default="1000,5000,10000,20000,50000", help="serve: arrival rates (queries/s)")
    ap.add_argument("--queries", type=int, default=4000, help="serve: queries per rate")
    ap.add_argument("--warmup-queries", type=int, default=400, help="serve: leading queries left out of the stats")
    ap.add_argument("--server-config", default="", help='serve: JSON object of bfs_server_create arguments, e.g. {"num_streams": 8}')
    return ap.parse_args()


def main() -> int:
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(batched and served BFS would shard by replicating each graph on every GPU)",
              file=sys.stderr)
        return 2
    if args.batch_case:
        name, _, width = args.batch_case.partition(":")
        if args.mode != "batch" or name not in ("rmat22", "er22_d16") or not width.isdigit() or \
                not 1 <= int(width) <= 64:
            print(f"--batch-case wants --mode batch and rmat22:B or er22_d16:B with B in 1..64, "
                  f"not {args.batch_case!r}", file=sys.stderr)
            return 2

    import torch

    import graphgen
    import paper_1604_02844_amd as bfs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    bfs.load_library()
    if args.mode == "batch":
        return bench_batch(args)
    if args.mode == "ceilings":
        return bench_ceilings(args)
    if args.mode == "serve":
        return bench_serve(args)

    t_gen = time.perf_counter()
    g = graphgen.cached("rmat", scale=args.scale, edgefactor=args.edgefactor, seed=args.seed)
    roots = graphgen.pick_roots(g, args.roots, seed=args.root_seed)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] graph {g.name}: n={g.n} nnz={g.nnz} ({t_gen:.1f}s), {len(roots)} roots", file=sys.stderr,
          flush=True)
    dg = bfs.bfs_graph_load_csr(g.offsets_i32() if args.offsets_i32 else g.offsets, g.cols,
                                bfs.BFS_LOAD_SYMMETRIC if args.hybrid else 0)
    run_flags = bfs.BFS_HYBRID if args.hybrid else 0
    # The autotuner's choice for this configuration, when one is shipped.
    from paper_1604_02844_amd import tune

    shipped = None if args.no_shipped_tunables else tune.apply_shipped(dg, "rmat", 0)
    if shipped:
        print(f"[bench] shipped autotuner tunables {shipped['key']}", file=sys.stderr, flush=True)
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
            st = bfs.bfs_run(dg, int(r), lv, pa, stream=stream, flags=run_flags)
            recs.append((int(r), st))
        return recs

    if args.copy_calibration > 0:
        # A plain elementwise copy of known size: the yardstick that scales the
        # FETCH_SIZE / WRITE_SIZE counters of the BFS kernels to bytes.
        src = torch.zeros(args.copy_calibration // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.add(src, 1, out=dst)
        torch.cuda.synchronize()
        del src, dst

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
    hyb_bytes = {}
    if args.hybrid:
        # Direction-optimising runs: bytes from each root's levels (an untimed
        # rerun after the timed region; levels are the same every run).
        deg = torch.from_numpy(np.diff(g.offsets)).to(dev)
        for r in roots:
            bfs.bfs_run(dg, int(r), lv, pa, stream=stream, flags=run_flags)
            hyb_bytes[int(r)] = hybrid_algorithmic_bytes(lv, deg, off_bytes)
        del deg
    inv_teps = 0.0
    bytes_total = 0
    ms_total = 0.0
    per_root = []
    for r, st in all_recs:
        t = st["device_ms"] * 1e-3
        m = st["edges_traversed"]
        inv_teps += t / m if m > 0 else float("inf")
        b = hyb_bytes[r] if args.hybrid else algorithmic_bytes(g.n, st["reached"], st["arcs_scanned"],
                                                                 st["num_levels"], off_bytes)
        bytes_total += b
        ms_total += st["device_ms"]
        per_root.append({"root": r, "ms": st["device_ms"], "m": m, "reached": st["reached"],
                         "arcs": st["arcs_scanned"], "levels": st["num_levels"], "bytes_alg": b,
                         "gteps": m / t / 1e9 if t > 0 else None})
    hm_gteps = len(all_recs) / inv_teps / 1e9 if inv_teps > 0 else 0.0
    launches = len(all_recs)
    avg_ms = ms_total / launches
    achieved = (bytes_total / launches) / (avg_ms * 1e-3) / 1e9

    from paper_1604_02844_amd import profsum

    workload_key = (f"rmat{args.scale} ef{args.edgefactor} seed{args.seed} roots{len(roots)} rootseed{args.root_seed} "
                    f"off{off_bytes * 8} tunables{args.tunables or '{}'}{' tuned' if args.tune else ''}"
                    f"{' hybrid' if args.hybrid else ''}")
    traffic = profsum.stored_traffic(
        os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                     f"bfs_run_rmat{args.scale}{'_hybrid' if args.hybrid else ''}_hbm_traffic.md"),
        workload_key)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        # The oracle as it stands: one serial queue BFS per host thread, on
        # every CPU this process may use up to the host share of one GPU, over
        # groups of the same roots (in order, wrapping) until at least
        # cpu_seconds of single-core work.
        info = host_info()
        threads = max(1, min(info["usable_cpus"], args.cpu_threads))
        res_all, cwall, used, cpu_s, at = [], 0.0, 0, 0.0, 0
        while cpu_s < args.cpu_seconds and len(res_all) < 64 * len(roots):
            group = [roots[(at + i) % len(roots)] for i in range(threads)]
            at += threads
            res, w, used = oracle.bfs_many(g.offsets, g.cols, group, threads=threads)
            res_all += res
            cwall += w
            cpu_s += sum(t for _, t, _ in res)
        inv = sum(t / s["edges"] for _, t, s in res_all if s["edges"] > 0)
        cpu = {"value": round(len(res_all) / inv / 1e9, 4) if inv > 0 else 0.0,
               "unit": "GTEPS (harmonic mean over roots)", "cores": used, "kind": "oracle",
               "sample": f"{len(res_all)} serial queue BFS runs from the first roots of the same {len(roots)}, "
                         f"{cpu_s:.1f} s of single-core work on {used} threads ({cwall:.2f} s wall); "
                         f"value = harmonic mean of per-run TEPS on one core; threads = the CPUs this process "
                         f"may use, at most {args.cpu_threads} (the host share of one GPU)",
               "throughput_gteps": round(sum(s["edges"] for _, _, s in res_all) / cwall / 1e9, 4),
               "roots_per_s": round(len(res_all) / cwall, 3), "host": info}

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
        "config": {"workload": f"single-root {'direction-optimising (top-down + bottom-up)' if args.hybrid else 'top-down'} "
                               f"BFS, R-MAT scale {args.scale}, edgefactor {args.edgefactor}, "
                               f"A/B/C/D=.57/.19/.19/.05, permuted, symmetrised, deduplicated, int32 cols, "
                               f"int{off_bytes * 8} offsets, {len(roots)} seeded roots of degree>0",
                   "n": g.n, "nnz": g.nnz, "roots": len(roots), "step": f"{len(roots)} BFS runs",
                   "tunables": bfs.bfs_graph_get_tunables(dg),
                   "tunables_from": ("autotuner, shipped cache " + shipped["key"]) if shipped and not args.tunables
                   else ("--tunables" if args.tunables else "library defaults")},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "bfs_run: k_init, k_expand + k_restore per level, k_out on the degree-ordered copy",
                     "avg_launch_ms": round(avg_ms, 4), "bytes_alg_per_launch": int(bytes_total / launches),
                     "workload_key": workload_key,
                     **({"bytes_model": "per level, the cheaper direction's compulsory reads (a lower bound "
                                        "for any choice of directions); see hybrid_algorithmic_bytes"}
                        if args.hybrid else {})},
        "cpu_baseline": cpu,
    }
    if not args.no_batch:
        del dg, lv, pa
        torch.cuda.empty_cache()
        out["batch"] = batch_case(args, "rmat22", 64, max(args.steps, 1))
    if args.details:
        with open(args.details, "w") as f:
            json.dump({"per_root": per_root, "summary": out}, f, indent=1)
    print(json.dumps(out), flush=True)
    return 0


def _single_times(bfs, dg, roots, lv, pa):
    out = []
    for r in roots:
        st = bfs.bfs_run(dg, int(r), lv, pa)
        out.append((st["device_ms"], st["edges_traversed"]))
    return out


def _batch_graph(name: str, seed: int):
    import graphgen

    if name == "rmat22":
        return graphgen.cached("rmat", scale=22, edgefactor=16, seed=seed)
    if name == "er22_d16":
        return graphgen.cached("er", n=1 << 22, avg_degree=16, seed=seed)
    raise ValueError(name)


def batch_case(args, name: str, widths, steps: int, other_form: bool = True):
    """Multi-source runs of the first `b` seeded roots for each width b, against
    the same roots run one at a time. Per case: the mean device time of `steps`
    batch runs (after one untimed run), aggregate GTEPS, the algorithmic bytes
    of one batch run and its roofline fraction. Returns one record, or a list
    when `widths` is a list."""
    import torch

    import graphgen
    import paper_1604_02844_amd as bfs

    one = not isinstance(widths, (list, tuple))
    widths = [widths] if one else list(widths)
    g = _batch_graph(name, args.seed)
    dg = bfs.bfs_graph_load_csr(g.offsets, g.cols)
    from paper_1604_02844_amd import tune

    shipped = None if args.no_shipped_tunables else tune.apply_shipped(dg, "rmat" if name.startswith("rmat") else "er", 1)
    deg = torch.from_numpy(np.diff(g.offsets)).cuda()
    pool = graphgen.pick_roots(g, max(widths), seed=args.root_seed)
    lv1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa1 = torch.empty(g.n, dtype=torch.int32, device="cuda")
    _single_times(bfs, dg, pool[:2], lv1, pa1)  # warm-up
    single = _single_times(bfs, dg, pool, lv1, pa1)
    del lv1, pa1
    print(f"[bench] {name}: n={g.n} nnz={g.nnz}, single-root runs done", file=sys.stderr, flush=True)
    results = []
    for b in widths:
        lv = torch.empty((b, g.n), dtype=torch.int32, device="cuda")
        pa = torch.empty((b, g.n), dtype=torch.int32, device="cuda")
        # The other launch form first (per-level launches when the default is
        # one persistent launch, or the reverse), for comparison only.
        t_other = None
        form = bfs.bfs_graph_get_tunables(dg)["persistent"]
        if other_form:
            bfs.bfs_graph_set_tunables(dg, persistent=-form)
            bfs.bfs_run_batch(dg, pool[:b], lv, pa)
            t_other = sum(bfs.bfs_run_batch(dg, pool[:b], lv, pa)["device_ms"] for _ in range(steps)) / steps
            bfs.bfs_graph_set_tunables(dg, persistent=form)
        bfs.bfs_run_batch(dg, pool[:b], lv, pa)  # warm-up
        sts = [bfs.bfs_run_batch(dg, pool[:b], lv, pa) for _ in range(steps)]
        t_ms = sum(st["device_ms"] for st in sts) / len(sts)
        st = sts[-1]
        m_sum = sum(m for _, m in single[:b])
        t_single = sum(t for t, _ in single[:b])
        assert st["edges_traversed"] == m_sum, (st, m_sum)
        rows, row_arcs = batch_active_rows(lv, deg, st["num_levels"])
        b_alg = batch_algorithmic_bytes(g.n, b, st["num_levels"], rows, row_arcs, st["reached"], 8)
        achieved = b_alg / (t_ms * 1e-3) / 1e9
        rec = {"graph": name, "n": g.n, "nnz": g.nnz, "roots": b, "batch_ms": round(t_ms, 3),
               "batch_gteps": round(m_sum / (t_ms * 1e-3) / 1e9, 2),
               "one_at_a_time_ms": round(t_single, 3),
               "one_at_a_time_gteps": round(m_sum / (t_single * 1e-3) / 1e9, 2),
               "levels": st["num_levels"], "active_rows": rows, "active_row_arcs": row_arcs,
               "bytes_alg": b_alg, "achieved_gbs": round(achieved, 1),
               "frac": round(achieved / HBM_PEAK_GBS, 4), "runs": len(sts),
               "launch": "one cooperative launch for all levels" if form > 0 else "one launch per kernel and level",
               "tunables_from": ("autotuner, shipped cache " + shipped["key"]) if shipped else "library defaults",
               "other_launch_form_ms": round(t_other, 3) if t_other is not None else None}
        rec["speedup"] = round(rec["batch_gteps"] / rec["one_at_a_time_gteps"], 2)
        results.append(rec)
        print(f"[bench] {rec}", file=sys.stderr, flush=True)
        del lv, pa
    del dg, deg
    torch.cuda.empty_cache()
    return results[0] if one else results


def bench_batch(args) -> int:
    results = []
    if args.batch_case:  # checked in main
        name, _, width = args.batch_case.partition(":")
        results += batch_case(args, name, [int(width)], max(args.steps, 1), other_form=False)
    else:
        for name, widths in (("rmat22", [64]), ("er22_d16", [8, 32, 64])):
            results += batch_case(args, name, widths, max(args.steps, 1))
    head = results[0]
    out = {"metric": "batched multi-source GTEPS (aggregate) vs one root at a time", "value": head["batch_gteps"],
           "unit": "GTEPS", "n_gpus": 1, "steps": args.steps, "higher_is_better": True, "dtype": "int32",
           "data": "synthetic", "config": {"workload": "multi-source BFS, 64-bit bit-sliced masks; R-MAT scale 22 "
                                                       "(64 roots) and Erdos-Renyi 2^22 avg degree 16 (8/32/64 roots)"},
           "roofline": {"bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": head["frac"], "traffic": None,
                        "kernel": f"bfs_run_batch ({head['launch']}), {head['graph']}, {head['roots']} roots",
                        "bytes_alg_per_launch": head["bytes_alg"]},
           "cases": results}
    print(json.dumps(out), flush=True)
    return 0


def _serve_graphs(seed):
    import graphgen

    specs = [("rmat16", dict(scale=16)), ("rmat18", dict(scale=18)), ("rmat20", dict(scale=20)),
             ("rmat22", dict(scale=22)), ("rmat24", dict(scale=24)),
             ("er18_d8", dict(n=1 << 18, avg_degree=8)), ("er20_d16", dict(n=1 << 20, avg_degree=16)),
             ("er22_d32", dict(n=1 << 22, avg_degree=32))]
    out = []
    for name, kw in specs:
        if name.startswith("rmat"):
            g = graphgen.cached("rmat", edgefactor=16, seed=seed, **kw)
        else:
            g = graphgen.cached("er", seed=seed, **kw)
        out.append((name, g))
    return out


def _trace(graphs, rate, count, seed):
    """Poisson arrivals (seconds), Zipf(1.1) graph choice over ranks 1..8, roots
    uniform over the chosen graph's vertices of degree > 0."""
    import graphgen

    gaps = -np.log1p(-graphgen.uniform_f64(seed, 30 + int(rate) % 997, count)) / rate
    arrivals = np.cumsum(gaps)
    w = np.array([k ** -1.1 for k in range(1, len(graphs) + 1)])
    cdf = np.cumsum(w / w.sum())
    choice = np.searchsorted(cdf, graphgen.uniform_f64(seed + 1, 40 + int(rate) % 997, count), side="right")
    choice = np.minimum(choice, len(graphs) - 1)
    pools = [np.nonzero(np.diff(g.offsets) > 0)[0] for _, g in graphs]
    pick = graphgen.uniform_u64(seed + 2, 50 + int(rate) % 997, count, 1 << 62)
    roots = np.array([pools[c][int(pick[i] % len(pools[c]))] for i, c in enumerate(choice)], dtype=np.int64)
    return arrivals, choice, roots


def bench_ceilings(args) -> int:
    """Memory-system ceilings (libceilings.so): streaming read and copy of 1 GiB,
    random 4-byte gathers from tables of 128 KiB to 128 MiB (8 gathers in flight
    per thread), random device-scope atomicOr without a returned value into a
    2 MiB table, and back-to-back empty launches. One JSON line."""
    import ctypes

    import torch

    lib = ctypes.CDLL(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1604_02844_amd",
                                   "libceilings.so"))
    i64, i32, vp, pf = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_float)
    lib.ceil_read.argtypes = [vp, i64, vp, i32, pf]
    lib.ceil_copy.argtypes = [vp, vp, i64, i32, pf]
    lib.ceil_gather.argtypes = [vp, i64, i64, vp, i32, pf]
    lib.ceil_atomic_or.argtypes = [vp, i64, i64, i32, pf]
    lib.ceil_empty.argtypes = [i32, pf]
    ms = ctypes.c_float()

    def call(fn, *a):
        rc = fn(*a, ctypes.byref(ms))
        if rc != 0:
            raise RuntimeError(f"{fn.__name__} returned {rc}")
        return ms.value

    gib = 1 << 30
    src = torch.ones(gib // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = {"metric": "memory-system ceilings", "n_gpus": 1, "data": "synthetic"}
    t = call(lib.ceil_read, src.data_ptr(), gib, sink.data_ptr(), 10)
    out["stream_read_gbs"] = round(gib / (t * 1e-3) / 1e9, 1)
    t = call(lib.ceil_copy, dst.data_ptr(), src.data_ptr(), gib, 10)
    out["copy_gbs"] = round(2 * gib / (t * 1e-3) / 1e9, 1)
    gathers = {}
    count = 1 << 28
    for kib in (128, 2048, 8192, 32768, 131072):
        words = kib * 256
        t = call(lib.ceil_gather, src.data_ptr(), words, count, sink.data_ptr(), 5)
        gathers[f"{kib}KiB"] = round(count / (t * 1e-3) / 1e9, 1)
    out["random_gather_g_per_s"] = gathers
    table = torch.zeros(1 << 19, dtype=torch.int32, device="cuda")
    count = 1 << 26
    t = call(lib.ceil_atomic_or, table.data_ptr(), 1 << 19, count, 5)
    out["atomic_or_2MiB_g_per_s"] = round(count / (t * 1e-3) / 1e9, 1)
    t = call(lib.ceil_empty, 1000)
    out["empty_launch_us"] = round(t * 1e3, 2)
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args) -> int:
    import threading

    import torch

    import paper_1604_02844_amd as bfs

    graphs = _serve_graphs(args.seed)
    dgs = [bfs.bfs_graph_load_csr(g.offsets, g.cols) for _, g in graphs]
    print(f"[bench] serving graphs loaded: {[(nm, g.n, g.nnz) for nm, g in graphs]}", file=sys.stderr, flush=True)
    rates = [float(x) for x in args.rates.split(",")]
    per_rate = []
    lv1 = {i: torch.empty(g.n, dtype=torch.int32, device="cuda") for i, (_, g) in enumerate(graphs)}
    pa1 = {i: torch.empty(g.n, dtype=torch.int32, device="cuda") for i, (_, g) in enumerate(graphs)}
    for rate in rates:
        arrivals, choice, roots = _trace(graphs, rate, args.queries, 3)
        # --- continuous-batching server
        srv = bfs.bfs_server_create(**(json.loads(args.server_config) if args.server_config else {}))
        gids = [bfs.bfs_server_add_graph(srv, d) for d in dgs]
        tickets = [None] * args.queries
        done = {}

        def submitter():
            t0 = time.perf_counter()
            for i in range(args.queries):
                delay = arrivals[i] - (time.perf_counter() - t0)
                if delay > 0.0002:
                    time.sleep(delay)
                tickets[i] = bfs.bfs_server_submit(srv, gids[choice[i]], int(roots[i]))

        th = threading.Thread(target=submitter)
        t_start = time.perf_counter()
        th.start()
        pending = 0
        while len(done) < args.queries:
            progressed = False
            for i in range(pending, args.queries):
                if tickets[i] is None:
                    break
                if i in done:
                    continue
                st = bfs.bfs_server_poll(srv, tickets[i])
                if st is not None:
                    done[i] = st
                    progressed = True
            while pending in done:
                pending += 1
            if not progressed:
                time.sleep(0.0002)
        t_end = time.perf_counter()
        th.join()
        bfs.bfs_server_destroy(srv)
        lat = np.array([done[i]["latency_ms"] for i in range(args.warmup_queries, args.queries)])
        m_total = sum(done[i]["edges_traversed"] for i in range(args.queries))
        # --- the same trace through single-root runs, FIFO, one at a time
        fifo_lat = []
        t0 = time.perf_counter()
        for i in range(args.queries):
            now = time.perf_counter() - t0
            if arrivals[i] > now:
                time.sleep(arrivals[i] - now)
            c = int(choice[i])
            bfs.bfs_run(dgs[c], int(roots[i]), lv1[c], pa1[c])
            fifo_lat.append((time.perf_counter() - t0 - arrivals[i]) * 1e3)
        t_fifo = time.perf_counter() - t0
        fifo_lat = np.array(fifo_lat[args.warmup_queries:])
        rec = {"rate_qps": rate, "queries": args.queries,
               "server_p50_ms": round(float(np.percentile(lat, 50)), 3),
               "server_p99_ms": round(float(np.percentile(lat, 99)), 3),
               "server_gteps": round(m_total / (t_end - t_start) / 1e9, 3),
               "fifo_p50_ms": round(float(np.percentile(fifo_lat, 50)), 3),
               "fifo_p99_ms": round(float(np.percentile(fifo_lat, 99)), 3),
               "fifo_gteps": round(m_total / t_fifo / 1e9, 3)}
        # Where the server's time goes: latency per graph and path (after warm-up).
        rec["server_batched_share"] = round(float(np.mean([done[i]["batched"] for i in range(args.warmup_queries,
                                                                                              args.queries)])), 3)
        by_graph = {}
        for i in range(args.warmup_queries, args.queries):
            d = by_graph.setdefault(graphs[int(choice[i])][0], {"batched": [], "single": []})
            d["batched" if done[i]["batched"] else "single"].append(done[i]["latency_ms"])
        rec["server_by_graph"] = {
            name: {path: {"n": len(v), "p50_ms": round(float(np.percentile(v, 50)), 2),
                          "p99_ms": round(float(np.percentile(v, 99)), 2)}
                   for path, v in d.items() if v}
            for name, d in by_graph.items()}
        per_rate.append(rec)
        print(f"[bench] {rec}", file=sys.stderr, flush=True)
    best = max(per_rate, key=lambda r: r["server_gteps"])
    out = {"metric": "served BFS: aggregate GTEPS and p50/p99 latency per arrival rate", "value": best["server_gteps"],
           "unit": "GTEPS", "n_gpus": 1, "higher_is_better": True, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "8 resident graphs (R-MAT 16/18/20/22/24, ER 2^18 d8, 2^20 d16, 2^22 d32), "
                                  "Poisson arrivals, Zipf(1.1) graph choice, uniform roots of degree>0",
                      "warmup_queries": args.warmup_queries,
                      "server_config": json.loads(args.server_config) if args.server_config else {}},
           "rates": per_rate}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
