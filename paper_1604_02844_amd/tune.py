"""JSON cache around ``bfs_autotune``.

Tuned tunables are stored per (GPU architecture, graph family, scale bucket,
mode) in ``$BFS_TUNE_CACHE`` (default ``~/.cache/bfs_mi355x_tune.json``); a hit
applies the stored tunables, a miss runs the autotuner on the given sample roots
and records the result.
"""
from __future__ import annotations

import json
import math
import os

from . import bfs_autotune, bfs_graph_set_tunables


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


def tuned(dg, roots, family: str, mode: int = 0, retune: bool = False) -> dict:
    """Apply cached tunables for this graph class, tuning on ``roots`` on a miss."""
    path = cache_path()
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
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
