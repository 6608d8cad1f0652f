import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C ABI)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


def node_coords(n, L):
    """Node coordinates of a box of side L centred on the origin, arrays indexed [k, j, i]."""
    h = L / (n - 1)
    c = -0.5 * L + h * np.arange(n)
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    return X, Y, Z


def interior(a):
    return a[1:-1, 1:-1, 1:-1]


@pytest.fixture
def coords():
    return node_coords
