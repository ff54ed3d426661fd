import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def qc_lib():
    """The HIP library through its binding, on device 0 (GPU tests only)."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2412_10072_amd import qc
    return qc.Context(0)
