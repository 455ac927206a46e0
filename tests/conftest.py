import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def gpu():
    """Skip only where no GPU exists at all; on a GPU host a missing or
    broken HIP library is an error, not a skip."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU on this host")
    from paper_1305_5120_amd import chfsi
    chfsi.load()  # raises if the HIP library is absent
    return torch.device("cuda:0")


@pytest.fixture(scope="session")
def lib(gpu):
    """The Python binding of the HIP library (loaded by the gpu fixture)."""
    from paper_1305_5120_amd import chfsi
    return chfsi
