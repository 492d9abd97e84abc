import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD GPU (MI355X) and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle test")


@pytest.fixture(scope="session", autouse=True)
def _built_oracle():
    """Build the CPU oracle if it is not built or older than its sources (test infrastructure)."""
    from oracle import build as ob
    if not os.path.exists(ob.LIB) or os.path.getmtime(ob.LIB) < max(os.path.getmtime(s) for s in ob.SRCS):
        ob.build()
