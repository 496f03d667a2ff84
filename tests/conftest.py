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
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")


@pytest.fixture
def progress(capsys):
    """Print a progress line past pytest's output capture, so that a long GPU
    test shows it is alive even when run without -s."""
    def say(*args, **kw):
        kw["flush"] = True
        with capsys.disabled():
            print(*args, **kw)
    return say
