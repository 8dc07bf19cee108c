import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running oracle case")


@pytest.fixture(scope="session")
def orc_small():
    """Toy parameters: N=64, 4 x 30-bit primes, 2 special primes, dnum 2."""
    from oracle import pyoracle as P
    return P.Oracle(6, 4, 30, 2, 31, 2, 20, 11)
