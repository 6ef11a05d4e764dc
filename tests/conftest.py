import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


def ensure_library():
    """Build liblbrr.so in-tree if (and only if) it is not there yet."""
    from paper_1505_06900_amd import build as _build

    if not os.path.exists(_build.LIB):
        _build.build()
    return _build.LIB


@pytest.fixture(scope="session")
def lbrr():
    ensure_library()
    import paper_1505_06900_amd as P

    return P


@pytest.fixture(scope="session")
def gpu(lbrr):
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")
    return torch
