import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    """The C oracle, built on first use if the library is not there yet."""
    from oracle import oracle as o
    if not os.path.exists(o.LIB):
        o.build()
    return o


@pytest.fixture(scope="session")
def lib():
    """The HIP library's Python binding; GPU tests only."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_07980_amd import ocsr
    ocsr.load()   # raises when the built library is missing
    return ocsr
