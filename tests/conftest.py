import os
import sys

import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_ctx():
    """One library context on cuda:0 for the GPU tests (fails loudly if the HIP
    library is not built)."""
    import torch
    from paper_1204_0069_amd import Context
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    ctx = Context(0)
    yield ctx
    ctx.close()
