import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")
    config.addinivalue_line("markers", "slow: long-running (large workloads)")
    config.addinivalue_line("markers", "cpu: runs on the host only")


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel(a, b):
    """max_i |a_i - b_i| / max_i |b_i| (element by element, scaled by the largest value)."""
    import numpy as np
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def parity_err(a, b):
    """Error figure of a parity check: max(relative L2, per-element error / 10).

    `parity_err(a, b) < tol` holds when ||a - b||_2 / ||b||_2 < tol AND every element
    satisfies |a_i - b_i| < 10 tol max_j |b_j|, so a fault confined to a few tiles, FFT
    lines or near blocks cannot hide under the norm of millions of correct values."""
    return max(rel_l2(a, b), 0.1 * max_rel(a, b))


@pytest.fixture(scope="session")
def o1():
    from oracle import direct
    return direct
