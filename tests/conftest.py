import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU oracle check")


def rel_err(a, b):
    """Normwise and max-wise relative error of a against reference b (complex as pairs)."""
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    mb = np.abs(b).max()
    if nb == 0:
        return float(np.abs(a).max())
    return max(np.linalg.norm((a - b).ravel()) / nb, np.abs(a - b).max() / mb)


@pytest.fixture
def relerr():
    return rel_err
