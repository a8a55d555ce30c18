import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: large inputs; still CPU-only unless also marked gpu")


@pytest.fixture(autouse=True)
def _gpu_progress(request):
    """GPU tests announce themselves before they touch the device (flushed), so a
    slow case is never silent and a failing one is named in the log."""
    if request.node.get_closest_marker("gpu") is None:
        yield
        return
    import time

    print(f"\n[gpu-test] start {request.node.nodeid}", flush=True)
    t0 = time.time()
    yield
    print(f"[gpu-test] end {request.node.nodeid} {time.time() - t0:.2f}s", flush=True)
