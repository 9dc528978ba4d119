"""Shared pytest configuration: the ``gpu`` marker, repo-root imports, and
seeded test primes drawn with sympy (a third-party primality routine, so
neither the oracle nor the library under test chooses its own inputs)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU test")


def test_primes(lo: int, hi: int, count: int, seed: int) -> list[int]:
    """``count`` distinct primes drawn uniformly from [lo, hi) (seeded)."""
    import sympy

    rng = np.random.default_rng(seed)
    out: list[int] = []
    seen = set()
    while len(out) < count:
        q = int(sympy.nextprime(int(rng.integers(lo, hi)) - 1))
        if lo <= q < hi and q not in seen:
            seen.add(q)
            out.append(q)
    return out


test_primes.__test__ = False  # a helper, not a test


@pytest.fixture
def primes():
    return test_primes
