import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def ctx():
    """A library context on cuda:0 bound to torch's current stream.  GPU tests
    fail loudly (no fallback) when the HIP library is missing."""
    if not gpu_available():
        pytest.skip("no GPU visible")
    from paper_2601_16734_amd import binding
    c = binding.Context(0)
    yield c
    c.close()
