import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle
    if not os.path.exists(oracle.LIB) or os.path.getmtime(oracle.LIB) < os.path.getmtime(oracle.SRC):
        oracle.build(force=True)
    yield


def pytest_runtest_logstart(nodeid, location):
    # one line per test as it starts, so a long GPU run shows where it is
    import sys
    import time
    sys.stderr.write(f"[{time.strftime('%H:%M:%S')}] start {nodeid}\n")
    sys.stderr.flush()
