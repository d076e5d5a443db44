import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def vms_lib():
    """The built HIP library's binding; GPU tests fail loudly when it is missing."""
    if not gpu_available():
        pytest.fail("GPU test collected without a visible HIP device")
    from paper_0809_4802_amd import binding
    return binding
