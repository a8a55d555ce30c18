"""Text summaries of rocprofv3 CSV output for the BFS kernels.

    python -m paper_1604_02844_amd.profsum trace DIR --runs N [--title T] [--command C]
                                                  [--kernels K1,K2,...] [--unit U]
        per-kernel calls, total and average duration from the kernel trace
        (rocprofv3 --kernel-trace --stats --output-format csv -d DIR), and the
        kernel time per BFS run (or per U, over the kernels K).
    python -m paper_1604_02844_amd.profsum traffic FETCH_DIR WRITE_DIR --runs N --copy-bytes B ...
        HBM traffic per BFS run from two counter passes (--pmc FETCH_SIZE, then
        --pmc WRITE_SIZE), each scaled by what the same counter reads for the
        plain copy kernel of B bytes in the same process.

The digest of the sources of the single-root kernels is written into every
summary; bench.py reports a stored traffic figure only while those sources
still match it.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
import shlex
import sys
from collections import defaultdict

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
# Kernels inside the span that bfs_run times (init, expand/restore per level,
# and on the degree-ordered copy the pass that writes the caller's arrays).
RUN_KERNELS = ("k_init", "k_expand", "k_restore", "k_out")
# Sources that define those kernels and the data they touch.
RUN_SOURCES = ("single.hip", "bfs_internal.h", "graph.cpp")
COPY_KERNEL_HINT = "_add<"  # torch.add(src, 1, out=dst): reads and writes every byte once


def source_digest() -> str:
    """sha256 over the sources of the single-root run's kernels (RUN_SOURCES)."""
    h = hashlib.sha256()
    for name in sorted(RUN_SOURCES):
        h.update(name.encode())
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def base_name(kernel: str) -> str:
    """'void bfs::k_expand<long, false>(bfs::SingleParams, int)' -> 'k_expand'."""
    m = re.search(r"(?:^|[\s:])(k_[A-Za-z0-9_]+)", kernel)
    if m:
        return m.group(1)
    name = kernel[5:] if kernel.startswith("void ") else kernel
    return name.split("(")[0].strip()[:100]


def _find(root: str, suffix: str) -> list[str]:
    return sorted(glob.glob(os.path.join(root, "**", f"*{suffix}"), recursive=True))


def _col(row: dict, *names: str) -> str:
    low = {k.lower(): v for k, v in row.items() if k}
    for n in names:
        if n.lower() in low:
            return low[n.lower()]
    raise KeyError(f"none of {names} in {list(row)}")


def read_trace(root: str) -> dict[str, list[int]]:
    """Kernel base name -> list of durations (ns)."""
    files = _find(root, "kernel_trace.csv")
    if not files:
        raise SystemExit(f"no *kernel_trace.csv under {root}")
    out: dict[str, list[int]] = defaultdict(list)
    for path in files:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                name = _col(row, "Kernel_Name", "KernelName", "Name")
                dur = int(_col(row, "End_Timestamp", "EndNs")) - int(_col(row, "Start_Timestamp", "BeginNs"))
                out[base_name(name)].append(dur)
    return out


def read_counter(root: str, counter: str) -> dict[str, list[float]]:
    """Kernel base name -> per-dispatch values of `counter`."""
    files = _find(root, "counter_collection.csv")
    if not files:
        raise SystemExit(f"no *counter_collection.csv under {root}")
    per: dict[tuple, float] = defaultdict(float)
    names: dict[tuple, str] = {}
    for path in files:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                if _col(row, "Counter_Name") != counter:
                    continue
                key = (path, _col(row, "Dispatch_Id", "Correlation_Id"))
                per[key] += float(_col(row, "Counter_Value"))
                names[key] = base_name(_col(row, "Kernel_Name"))
    out: dict[str, list[float]] = defaultdict(list)
    for key, v in per.items():
        out[names[key]].append(v)
    return out


def cmd_trace(a) -> None:
    tr = read_trace(a.dir)
    kernels = tuple(k for k in a.kernels.split(",") if k) if a.kernels else RUN_KERNELS
    unit = a.unit
    lines = [f"# {a.title}", "", f"Command: `{a.command}`", "", f"Summary: `{_self_command()}`", "",
             f"Library source digest: {source_digest()}",
             f"{unit[0].upper() + unit[1:]}{'es' if unit.endswith(('s', 'x', 'ch', 'sh')) else 's'} in the trace: "
             f"{a.runs}", "",
             "| kernel | calls | total ms | avg us | min us | max us |", "|---|---|---|---|---|---|"]
    total_run = 0.0
    for k, d in sorted(tr.items(), key=lambda kv: -sum(kv[1])):
        tot = sum(d)
        if k in kernels:
            total_run += tot
        lines.append(f"| {k} | {len(d)} | {tot / 1e6:.3f} | {tot / len(d) / 1e3:.2f} | {min(d) / 1e3:.2f} | "
                     f"{max(d) / 1e3:.2f} |")
    lines += ["", f"Kernel time per {unit} ({' + '.join(kernels)}): {total_run / a.runs / 1e6:.4f} ms"]
    for k in kernels:
        if k in tr:
            lines.append(f"  {k}: {sum(tr[k]) / a.runs / 1e6:.4f} ms per {unit}, "
                         f"{len(tr[k]) / a.runs:.1f} launches per {unit}")
    print("\n".join(lines))


def cmd_traffic(a) -> None:
    fetch = read_counter(a.fetch_dir, "FETCH_SIZE")
    write = read_counter(a.write_dir, "WRITE_SIZE")

    def copy_kib(c):
        vals = [v for k, vs in c.items() if COPY_KERNEL_HINT in k for v in vs]
        if not vals:
            raise SystemExit(f"no copy kernel ({COPY_KERNEL_HINT}) among {list(c)}")
        return max(vals)

    f_copy, w_copy = copy_kib(fetch), copy_kib(write)
    f_scale = a.copy_bytes / (f_copy * 1024.0)
    w_scale = a.copy_bytes / (w_copy * 1024.0)
    f_run = sum(sum(fetch.get(k, [])) for k in RUN_KERNELS) * 1024.0 * f_scale / a.runs
    w_run = sum(sum(write.get(k, [])) for k in RUN_KERNELS) * 1024.0 * w_scale / a.runs
    lines = [f"# {a.title}", "", f"Fetch pass: `{a.fetch_command}`", "", f"Write pass: `{a.write_command}`", "",
             f"Summary: `{_self_command()}`", "",
             f"Copy kernel: {a.copy_bytes} B read and written; FETCH_SIZE reads {f_copy:.0f} KiB "
             f"(scale {f_scale:.4f}), WRITE_SIZE reads {w_copy:.0f} KiB (scale {w_scale:.4f})",
             f"BFS runs per pass: {a.runs}", "",
             "| kernel | dispatches | FETCH KiB (raw) | WRITE KiB (raw) | scaled MB per run |", "|---|---|---|---|---|"]
    for k in sorted(set(fetch) | set(write)):
        fk, wk = sum(fetch.get(k, [])), sum(write.get(k, []))
        per = (fk * f_scale + wk * w_scale) * 1024.0 / a.runs / 1e6
        lines.append(f"| {k} | {len(fetch.get(k, []))} | {fk:.0f} | {wk:.0f} | {per:.3f} |")
    lines += ["", f"fetch_bytes_per_run: {int(f_run)}", f"write_bytes_per_run: {int(w_run)}",
              f"traffic_bytes_per_run: {int(f_run + w_run)}", f"workload: {a.workload}",
              f"source_digest: {source_digest()}"]
    print("\n".join(lines))


def _self_command() -> str:
    return "python -m paper_1604_02844_amd.profsum " + " ".join(shlex.quote(x) for x in sys.argv[1:])


def stored_traffic(path: str, workload: str) -> int | None:
    """traffic_bytes_per_run from a summary, if it was taken on `workload`
    with the current sources; else None."""
    try:
        with open(path) as f:
            text = f.read()
    except OSError:
        return None
    fields = dict(re.findall(r"^(\w+): (.+)$", text, flags=re.M))
    if fields.get("workload") != workload or fields.get("source_digest") != source_digest():
        return None
    try:
        return int(fields["traffic_bytes_per_run"])
    except (KeyError, ValueError):
        return None


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="profsum")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--runs", type=int, required=True)
    t.add_argument("--title", default="Kernel trace")
    t.add_argument("--command", default="")
    t.add_argument("--kernels", default="", help="comma-separated kernels counted per unit (default: a bfs_run's)")
    t.add_argument("--unit", default="BFS run", help="what --runs counts, for the labels")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--runs", type=int, required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--title", default="HBM traffic")
    c.add_argument("--fetch-command", default="")
    c.add_argument("--write-command", default="")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        cmd_trace(a)
    else:
        cmd_traffic(a)
    return 0


if __name__ == "__main__":
    sys.exit(main())
