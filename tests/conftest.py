import os
import sys

import pytest

# the oracle is OpenMP code: never spin-wait when cores are shared
os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    """Make sure the oracle shared library exists (gcc, CPU only)."""
    from oracle import build as ob
    if not os.path.exists(ob.LIB):
        ob.build()
    yield
