import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def have_gpu():
    import torch
    return torch.cuda.is_available()


@pytest.fixture(scope="session")
def lib():
    """The built C-ABI library (host-only calls need no GPU)."""
    path = os.path.join(ROOT, "paper_2009_06725_amd", "libscvs.so")
    if not os.path.exists(path):
        pytest.fail("libscvs.so is not built (run paper_2009_06725_amd/build.py)")
    from paper_2009_06725_amd import scvs
    return scvs.lib()
