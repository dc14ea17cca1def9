import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


import pytest  # noqa: E402


@pytest.fixture(scope="session")
def gauge32():
    """The benchmark's 32^3 x 64 gauge field (SU(3) parts and U(1) angles), generated once
    per test session for every full-size test."""
    from bench import DIMS, EPS, EPS_U1, SEED
    from paper_2202_07388_amd import synthetic as syn
    return syn.gauge_field(DIMS, EPS, EPS_U1, SEED)
