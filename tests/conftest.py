import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def tiny_problem():
    """One atom in a 4 bohr simple-cubic cell on an 8^3 grid (dense-diagonalisable)."""
    from workloads import custom_spec, make_problem
    spec = custom_spec("tiny", 90, 4.0, 1, 8, 512, 2.0, basis="sc", jitter_amp=0.2)
    return make_problem(spec)
