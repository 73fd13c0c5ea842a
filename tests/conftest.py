import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU-side setup (large trained forests)")


@pytest.fixture
def say(capsys):
    """Print a progress line past pytest's output capture, at once: long GPU
    tests (training the 1,024-tree forest takes minutes) must keep writing."""
    def _say(msg):
        with capsys.disabled():
            print(msg, flush=True)
    return _say
