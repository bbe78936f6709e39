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
def orc():
    import oracle
    oracle.lib()
    return oracle


@pytest.fixture
def report(capsys):
    """Print a line to the terminal even while pytest captures output (the
    replay counts of the full-size parity tests belong in the run's log)."""
    def emit(msg):
        with capsys.disabled():
            print(msg, flush=True)
    return emit
