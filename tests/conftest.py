import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs on the GPU box)")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def pair_ranks_n12d6():
    """The oracle's full pair map at n = 12, d = 6 (N x N int64, 2.8 GB;
    about half a minute of host time), shared by the full-size GPU tests."""
    import oracle as O
    return O.pair_ranks(12, 6)
