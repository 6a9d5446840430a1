import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


ORACLE_THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="session", autouse=True)
def _oracle_threads():
    """The oracle's block-tree loops run on the host's cores (results are the
    one-thread results bit for bit)."""
    import oracle
    oracle.build(force=False)
    oracle.set_threads(ORACLE_THREADS)


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


@pytest.fixture
def rng():
    return np.random.default_rng(1204)
