import os
import sys
import time

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(autouse=True)
def _progress_log(request):
    """Append each test id to gpurun_out/pytest_progress.log (when that folder
    exists) before the test runs, flushed, so a run that dies still names the
    case it was in."""
    out = os.path.join(ROOT, "gpurun_out")
    if os.path.isdir(out):
        with open(os.path.join(out, "pytest_progress.log"), "a") as fh:
            fh.write(f"{time.strftime('%H:%M:%S')} START {request.node.nodeid}\n")
            fh.flush()
            os.fsync(fh.fileno())
    yield
