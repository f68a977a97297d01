import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def cell256():
    """64-atom periodic diamond cell (2x2x2 conventional cells), M = 256, rng seed 0."""
    from paper_1307_3218_amd import lattice
    return lattice.workload("diamond_2x2x2")
