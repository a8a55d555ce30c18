"""JSON cache around ``bfs_autotune``.

Tuned tunables are stored per (GPU architecture, graph family, scale bucket,
mode) in ``$BFS_TUNE_CACHE`` (default ``~/.cache/bfs_mi355x_tune.json``); a hit
applies the stored tunables, a miss runs the autotuner on the given sample roots
and records the result.

``tuned_mi355x.json`` beside this file holds the autotuner's choices for the
benchmarked configurations, written by ``python -m paper_1604_02844_amd.tune
--ship`` on an MI355X (R-MAT scale 24 single-root on 8 roots, R-MAT scale 22
batched on 64 roots); ``apply_shipped`` applies an entry when one matches.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

from . import bfs_autotune, bfs_graph_set_tunables

SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_mi355x.json")


def cache_path() -> str:
    return os.environ.get("BFS_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "bfs_mi355x_tune.json"))


def _arch() -> str:
    try:
        import torch

        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def cache_key(family: str, n: int, mode: int) -> str:
    return f"{_arch()}|{family}|s{int(round(math.log2(max(n, 2))))}|m{mode}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned(dg, roots, family: str, mode: int = 0, retune: bool = False) -> dict:
    """Apply cached tunables for this graph class, tuning on ``roots`` on a miss."""
    path = cache_path()
    cache = _load(path)
    key = cache_key(family, dg.n, mode)
    if key in cache and not retune:
        return bfs_graph_set_tunables(dg, **cache[key])
    best = bfs_autotune(dg, roots, mode)
    cache[key] = best
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(path + ".tmp", path)
    except OSError:
        pass
    return best


def apply_shipped(dg, family: str, mode: int = 0):
    """Apply the shipped autotuner result for this graph class; None without one."""
    entry = _load(SHIPPED).get(cache_key(family, dg.n, mode))
    if entry is None:
        return None
    return {"key": cache_key(family, dg.n, mode), "tunables": bfs_graph_set_tunables(dg, **entry)}


def ship(path: str = SHIPPED) -> int:
    """Tune the benchmarked configurations and write the shipped cache to `path`."""
    import graphgen
    from . import bfs_graph_load_csr

    out = {}
    for scale, mode, roots_n, sample in ((24, 0, 64, 8), (22, 1, 64, 64)):
        g = graphgen.cached("rmat", scale=scale, edgefactor=16, seed=1)
        dg = bfs_graph_load_csr(g.offsets, g.cols)
        roots = graphgen.pick_roots(g, roots_n, seed=2)
        best = bfs_autotune(dg, roots[:sample], mode)
        out[cache_key("rmat", dg.n, mode)] = best
        print(f"rmat{scale} mode {mode}: {best}", file=sys.stderr, flush=True)
        del dg
    with open(path, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")
    return 0


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--ship", action="store_true", help="tune the benchmarked configurations (needs a GPU)")
    ap.add_argument("--out", default=SHIPPED, help="where to write the tuned cache")
    a = ap.parse_args()
    if a.ship:
        sys.exit(ship(a.out))
    ap.print_help()
