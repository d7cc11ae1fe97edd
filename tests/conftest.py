import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def oracle_pool():
    """One pool of host processes running the oracle's search, shared by
    the tests that check whole frames (see tests/parity.py)."""
    from tests.parity import OraclePool

    p = OraclePool()
    yield p
    p.close()
