import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X / gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def has_gpu() -> bool:
    try:
        import torch
        return bool(torch.cuda.is_available())
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its Python binding; fails loudly if the
    extension is missing (GPU tests must never fall back to anything)."""
    if not has_gpu():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_2206_13574_amd import gwfa
    return gwfa
