import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")


@pytest.fixture(scope="session")
def basis_c1():
    """Oracle basis of the 1500-point, l <= 2 single-centre workload (N = 86)."""
    from oracle.radial import BasisSpec, build_basis
    return build_basis(BasisSpec(n_max=3, l_max=2, n_bins=8, k_max=3.0, n_r=1500))


@pytest.fixture(scope="session")
def basis_small():
    """A small oracle basis for quick structural checks (bound n <= 3, 2 bins, l <= 2)."""
    from oracle.radial import BasisSpec, build_basis
    return build_basis(BasisSpec(n_max=3, l_max=2, n_bins=2, k_max=2.0, n_r=600))
