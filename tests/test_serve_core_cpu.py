"""The server's scheduling core on the CPU: tests/serve_core_fake.cpp drives
serve_core.h (the same core the C ABI's server runs on the GPU) with a host
engine, built with clang under ThreadSanitizer and under AddressSanitizer with
UndefinedBehaviorSanitizer. Scenarios: requests from several threads over four
graphs, few slots per instance, a memory budget that holds one instance and two
result rows, the single-root worker route, a device error after a few levels,
destroy with requests in flight, bad arguments. Each result is checked against
an independent queue BFS; a sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "serve_core_fake.cpp")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"


def _clang():
    if os.path.exists(CLANG):
        return CLANG
    found = shutil.which("clang++")
    if not found:
        pytest.skip("no clang++ with sanitizer runtimes")
    return found


@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_serve_core_under_sanitizer(tmp_path, sanitizer):
    exe = str(tmp_path / "serve_core_fake")
    cmd = [_clang(), "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           f"-fsanitize={sanitizer}", "-fno-sanitize-recover=all",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROOT, "paper_1604_02844_amd", "csrc"),
           SRC, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert "serve core: all scenarios ok" in out, out[-3000:]
    assert "Sanitizer" not in out, out[-6000:]
