import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libloopsplat.so")


@pytest.fixture(scope="session")
def gpu():
    """Skip unless a HIP device is present; returns the loaded binding."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_10154_amd import lib

    return lib.load()
