import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI on the device)")
    config.addinivalue_line("markers", "slow: oracle runs that take tens of seconds")


@pytest.fixture(scope="session")
def balib():
    """The device library (built first if no build exists)."""
    from paper_2510_15271_amd import ba, build_lib
    if not os.path.exists(ba.LIB_PATH):
        build_lib.build()
    return ba
