import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


_ORACLE_CACHE = {}


@pytest.fixture(scope="session")
def oracle_cache():
    """Oracle results shared across test modules within one run (the full
    256 x 256 x 128 gradient takes seconds of host time)."""
    return _ORACLE_CACHE
