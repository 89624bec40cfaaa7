import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def evx_gpu():
    """The HIP library bound through its C ABI, on cuda:0.  GPU tests fail (not skip) when the
    device or the built library is missing: a GPU run must exercise the native path."""
    import torch
    from paper_2507_21748_amd import evx
    assert torch.cuda.is_available(), "GPU test collected on a machine without a GPU"
    evx.load()
    return evx
