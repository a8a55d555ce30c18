"""bench.py's command-line contract that needs no GPU: more than one GPU is
refused with a message and exit status 2, before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, env=env)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="4")
    r = run_bench(env=env)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_bad_batch_case_is_refused():
    for bad in (["--mode", "batch", "--batch-case", "rmat99:64"], ["--mode", "batch", "--batch-case", "rmat22:65"],
                ["--mode", "batch", "--batch-case", "rmat22"], ["--batch-case", "rmat22:64"]):
        r = run_bench(*bad)
        assert r.returncode == 2, bad
        assert "--batch-case wants" in r.stderr
        assert r.stdout == ""
