import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


_capture = None


def pytest_configure(config):
    global _capture
    config.addinivalue_line("markers", "gpu: needs an AMD GPU and the built HIP library")
    _capture = config.pluginmanager.getplugin("capturemanager")


def progress(msg):
    """Print past pytest's output capture: a fixture that runs for minutes (full-size designs, training)
    shows each of its steps as it takes it, whatever the capture mode."""
    if _capture is not None:
        with _capture.global_and_fixture_disabled():
            print(msg, flush=True)
    else:
        print(msg, flush=True)


@pytest.fixture(scope="session")
def gpu_ctx():
    import torch
    import paper_1701_05936_amd as bl
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    ctx = bl.Context(0)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()
