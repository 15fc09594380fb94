import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def dwctx():
    """One library context on cuda:0 for all GPU tests."""
    import torch

    import paper_1204_5463_amd as P

    assert torch.cuda.is_available(), "GPU test needs an MI355X"
    ctx = P.Context(0)
    yield ctx
    ctx.close()
