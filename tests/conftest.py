import os
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# the autotuner's decisions of a test session go to a file of its own (read lazily by the library on
# its first lookup), so that no earlier run's cache decides which launch shapes a test exercises
os.environ.setdefault("HBJ_TUNE_CACHE", os.path.join(tempfile.gettempdir(), f"hbj_tune_test_{os.getpid()}.json"))


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def hbj():
    """The HIP-backed binding; fails loudly if the library is not built."""
    import paper_2209_10886_amd as hbj_mod

    return hbj_mod
