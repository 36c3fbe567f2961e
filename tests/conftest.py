import os
import sys

import pytest
import torch  # noqa: F401  (first import can be slow on a fresh box; pay it at collection)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library through its C-ABI binding; fails loudly when absent."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1704_02083_amd import rapid
    return rapid
