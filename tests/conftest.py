import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


@pytest.fixture(scope="session")
def kt():
    """The binding, with libkt.so built if (and only if) it is missing."""
    import paper_2008_13145_amd as kt
    if not os.path.exists(kt.LIB_PATH):
        from paper_2008_13145_amd import build
        build.build()
    return kt


@pytest.fixture(scope="session")
def gpu(kt):
    """A device handle on GPU 0 plus torch, for the parity tests."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    h = kt.Handle(0)
    yield h, torch
    torch.cuda.synchronize()
    h.close()
