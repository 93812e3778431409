import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C-ABI)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle import native
    native.lib()
    yield


@pytest.fixture(scope="session")
def ctx():
    """One library context on device 0 for all GPU tests."""
    from paper_2310_09204_amd import lib
    c = lib.Context(0)
    yield c
    c.close()
