import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test (still part of the CPU suite)")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library handle; the gpu tests fail (not skip) when it cannot be used."""
    import torch
    from paper_1411_0814_amd import _lib
    assert torch.cuda.is_available(), "gpu test run without a visible GPU"
    return _lib.lib()
