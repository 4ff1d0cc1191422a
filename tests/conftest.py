import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def solver():
    """One library context on cuda:0 for the whole GPU test session."""
    from paper_1906_10678_amd import msc

    s = msc.Solver(0, workspace_bytes=int(os.environ.get("MSC_TEST_WS_GB", "24")) << 30)
    yield s
    s.close()
