import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: statistical pin that takes tens of seconds")


@pytest.fixture(scope="session")
def orc():
    """The CPU oracle module (built on first use)."""
    from oracle import build as ob
    if not os.path.exists(ob.LIB):
        ob.build()
    from oracle import oracle as o
    return o


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
