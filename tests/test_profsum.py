"""profsum's trace summary on a synthetic rocprofv3 kernel trace (no GPU):
per-kernel rows, the per-unit kernel time over the chosen kernel set, and the
labels for a bfs_run trace and for a batch trace."""
import csv
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def write_trace(d, rows):
    os.makedirs(os.path.join(d, "host"), exist_ok=True)
    with open(os.path.join(d, "host", "1_kernel_trace.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        t = 1000
        for name, dur_ns in rows:
            w.writerow([name, t, t + dur_ns])
            t += dur_ns + 500


def summarise(d, *extra):
    r = subprocess.run([sys.executable, "-m", "paper_1604_02844_amd.profsum", "trace", d, *extra],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 0, r.stderr
    return r.stdout


def test_bfs_run_trace(tmp_path):
    d = str(tmp_path / "t")
    rows = []
    for _ in range(2):  # two runs: init, two expand/restore pairs, out
        rows += [("void bfs::(anonymous namespace)::k_init<long, 1024>(P, int)", 20_000),
                 ("void bfs::(anonymous namespace)::k_expand<long, 1024, false>(P, int)", 300_000),
                 ("void bfs::(anonymous namespace)::k_restore<long, false>(P, int)", 10_000),
                 ("void bfs::(anonymous namespace)::k_expand<long, 1024, false>(P, int)", 100_000),
                 ("void bfs::(anonymous namespace)::k_restore<long, false>(P, int)", 10_000),
                 ("bfs::(anonymous namespace)::k_out(R const*, int const*, int*, int*, long)", 70_000)]
    rows.append(("__amd_rocclr_copyBuffer", 5_000))
    write_trace(d, rows)
    out = summarise(d, "--runs", "2")
    assert "BFS runs in the trace: 2" in out
    assert "| k_expand | 4 | 0.800 | 200.00 | 100.00 | 300.00 |" in out
    assert "| __amd_rocclr_copyBuffer | 1 |" in out
    # (20 + 400 + 20 + 70) us per run; the copy is not a run kernel.
    assert "Kernel time per BFS run (k_init + k_expand + k_restore + k_out): 0.5100 ms" in out
    assert "k_expand: 0.4000 ms per BFS run, 2.0 launches per BFS run" in out


def test_batch_trace_kernel_set_and_unit(tmp_path):
    d = str(tmp_path / "b")
    rows = []
    for _ in range(4):
        rows += [("bfs::(anonymous namespace)::k_fill_i32(int*, long, int)", 150_000)] * 2
        rows += [("void bfs::(anonymous namespace)::k_ms_push<long, 256>(M, int)", 50_000),
                 ("void bfs::(anonymous namespace)::k_ms_pull<long>(M, int)", 1_000_000)]
    rows += [("void bfs::(anonymous namespace)::k_expand<long, 1024, false>(P, int)", 9_000_000)]
    write_trace(d, rows)
    out = summarise(d, "--runs", "4", "--unit", "batch", "--kernels", "k_fill_i32,k_ms_push,k_ms_pull")
    assert "Batches in the trace: 4" in out
    assert "Kernel time per batch (k_fill_i32 + k_ms_push + k_ms_pull): 1.3500 ms" in out
    assert "k_ms_pull: 1.0000 ms per batch, 1.0 launches per batch" in out
    assert "| k_expand | 1 | 9.000 |" in out  # listed, not counted per batch
