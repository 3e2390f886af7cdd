import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size (N=2^16, 24+8 primes) oracle cases")


@pytest.fixture(scope="session")
def params_small():
    """N=2^12, three 28-bit ciphertext primes, one 30-bit special prime (digit width 1)."""
    import oracle
    return oracle.Params(12, oracle.prime_chain(28, 12, 3), oracle.prime_chain(30, 12, 1))


@pytest.fixture(scope="session")
def params_full():
    """N=2^16, 24 ciphertext primes of 30 bits, 8 special primes of 31 bits (dnum 3)."""
    import oracle
    return oracle.Params(16, oracle.prime_chain(30, 16, 24), oracle.prime_chain(31, 16, 8))


@pytest.fixture(scope="session")
def params_mid():
    """N=2^13, 7 ciphertext primes of 30 bits, 3 special primes of 31 bits (ragged last digit)."""
    import oracle
    return oracle.Params(13, oracle.prime_chain(30, 13, 7), oracle.prime_chain(31, 13, 3))
