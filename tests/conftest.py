import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built libpmx.so")
    config.addinivalue_line("markers", "slow: takes more than ~20 s on the CPU")


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def pmx():
    """The ctypes binding of libpmx.so; GPU tests fail loudly when it is missing."""
    from paper_2603_09381_amd import pmx as mod
    mod.load()
    return mod
