import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def rng():
    import numpy as np
    return np.random.default_rng(12345)


@pytest.fixture(scope="session")
def px_ctx():
    """One library context on cuda:0 for all GPU tests (workspace reused)."""
    import torch
    from paper_2501_03061_amd import px
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    ctx = px.Context(0)
    yield ctx
    torch.cuda.synchronize()
    ctx.ws = None
    ctx.close()
