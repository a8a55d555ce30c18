"""Build libbfs.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1604_02844_amd.build [--force]
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbfs.so")
# Memory-system ceiling microbenchmarks (bench.py --mode ceilings): a library of their own.
CEIL_LIB = os.path.join(HERE, "libceilings.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
SOURCES = ["graph.cpp", "abi.cpp", "autotune.cpp", "server.cpp", "single.hip", "multi.hip", "parents.hip", "noalloc.hip"]
ARCH = os.environ.get("BFS_OFFLOAD_ARCH", "gfx950")

# Packed fp32 ops are disabled for all device code (no floating point is used on
# the device; the flag keeps the compiler from forming packed fp32 instructions).
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-result",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{INCLUDE}"]


def _needs(obj: str, deps: list[str]) -> bool:
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(force: bool = False, verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    headers = [os.path.join(CSRC, "bfs_internal.h"), os.path.join(CSRC, "serve_core.h"),
               os.path.join(INCLUDE, "bfs.h")]
    jobs = []
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OUT_DIR, src + ".o")
        objs.append(obj)
        if force or _needs(obj, [path] + headers):
            lang = ["-x", "hip"]
            jobs.append(["hipcc", *HIP_FLAGS, *lang, "-c", path, "-o", obj])

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{msg}")
        if verbose and msg.strip():
            print(msg)

    with ThreadPoolExecutor(max_workers=min(len(jobs), 8) or 1) as ex:
        list(ex.map(run, jobs))
    if force or jobs or _needs(LIB, objs):
        tmp = LIB + ".tmp"
        run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"])
        os.replace(tmp, LIB)
    ceil_src = os.path.join(CSRC, "ceilings.hip")
    if force or _needs(CEIL_LIB, [ceil_src]):
        tmp = CEIL_LIB + ".tmp"
        run(["hipcc", *HIP_FLAGS, "-shared", "-x", "hip", ceil_src, "-o", tmp])
        os.replace(tmp, CEIL_LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--force" in sys.argv, verbose=True))
