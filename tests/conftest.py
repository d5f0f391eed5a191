import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU and the built HIP library")


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
