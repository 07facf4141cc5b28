import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def small_dimer():
    """Water dimer, 60 points per atom (N = 360, P = 18)."""
    from paper_2208_14639_amd import inputs
    return inputs.make_problem(2, 60, 7)


@pytest.fixture(scope="session")
def tiny_problem():
    """One water, 8 points per atom (N = 24, P = 9)."""
    from paper_2208_14639_amd import inputs
    return inputs.make_problem(1, 8, 11)


@pytest.fixture(scope="session")
def becke_dimer():
    """Water dimer, 60 points per atom, Becke-partitioned weights with their
    first and second nuclear derivatives (N = 360, P = 18)."""
    from paper_2208_14639_amd import inputs
    return inputs.make_problem(2, 60, 7, weights="becke", weight_hessian=True)
