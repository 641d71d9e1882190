import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP) device")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def fft_poisson(q, h):
    """Exact periodic solution of M phi = -4 pi q / h by diagonalising the
    7-point stencil with the DFT: the eigenvalue of M for wave vector k is
    -sum_d 2 (1 - cos(2 pi k_d / N)); the k = 0 mode is set to zero (mean-zero
    gauge). A spectral method independent of the iterative oracle."""
    N = q.shape[0]
    k = np.arange(N)
    l1 = 2.0 * (1.0 - np.cos(2.0 * np.pi * k / N))
    lam = l1[:, None, None] + l1[None, :, None] + l1[None, None, :]
    lam[0, 0, 0] = 1.0
    ph = 4.0 * np.pi * np.fft.fftn(q) / (h * lam)
    ph[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(ph))


@pytest.fixture(scope="session")
def oracle_lib():
    import oracle
    oracle.build(force=False)
    return oracle
