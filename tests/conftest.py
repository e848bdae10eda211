import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def projector(E):
    """Orthogonal projector onto the span of the columns of E."""
    return E @ E.conj().T


def random_unitary(rng, n):
    Z = crandn(rng, n, n)
    Q, Rr = np.linalg.qr(Z)
    return Q * (np.diag(Rr) / np.abs(np.diag(Rr)))[None, :]


def random_pd(rng, M, cond=10.0):
    """Hermitian positive definite matrix with eigenvalues spread over [1, cond]."""
    Q = random_unitary(rng, M)
    ev = np.geomspace(1.0, cond, M)
    return (Q * ev[None, :]) @ Q.conj().T
