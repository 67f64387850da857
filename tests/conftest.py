import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library through its C ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def gpu():
    """The HIP library bound to cuda:0; GPU tests fail loudly if it cannot load."""
    import torch

    assert torch.cuda.is_available(), "GPU test needs a ROCm device"
    import paper_2405_08737_amd as kbe

    kbe.lib()  # raises if the shared library is missing
    return kbe
