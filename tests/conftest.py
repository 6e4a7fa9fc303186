import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_runtest_logstart(nodeid, location):
    """Name each test before it runs (flushed to a file), so a lost GPU run still says which case ran."""
    path = os.environ.get("IBM_TEST_PROGRESS")
    if path:
        with open(path, "a") as f:
            f.write(nodeid + "\n")
            f.flush()
            os.fsync(f.fileno())
