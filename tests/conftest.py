import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library)")


import functools

import pytest


@functools.lru_cache(maxsize=None)
def _oracle_gauss(J):
    from oracle.quadrature import gauss_legendre
    return gauss_legendre(J)


@pytest.fixture(scope="session")
def oracle_gauss():
    """The oracle's Gauss-Legendre latitudes, each J computed once per session
    (J = 1536 takes about half a minute in quad precision)."""
    return _oracle_gauss
