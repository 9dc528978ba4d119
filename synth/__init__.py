"""Seeded synthetic inputs shaped like the workloads of Dumas and Urbanska's
integer-determinant paper.

This module is shared by the CPU oracle and by the GPU path's tests and
benchmark.  It holds no arithmetic of the determinant method itself: it only
draws matrices, right-hand sides, sizes and arrival times from seeded
generators (numpy PCG64 via ``default_rng``), and builds matrices whose Smith
form is fixed by construction.

Workloads (Section 5.1, the experiments):
  * random dense matrices with entries uniform in a set of contiguous integers
    ({-8..8} in Fig. 1, {-100..100} in Fig. 2);
  * engineered matrices with the Smith form of diag(1, 2, ..., n) (Table 1);
  * matrices U*diag(s)*V with unimodular U, V and chosen invariant factors s,
    the shape that Section 3 analyses (several non-trivial invariant factors).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "dense_uniform",
    "batched_sizes",
    "unimodular_factors",
    "smith_matrix",
    "engineered_table1",
    "structured_serving",
    "random_rhs",
    "poisson_arrivals",
]


def dense_uniform(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """n x n int64 matrix, entries i.i.d. uniform in [lo, hi] (both ends
    included), drawn from ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=(n, n), dtype=np.int64)


def batched_sizes(count: int, n_min: int, n_max: int, seed: int) -> list[int]:
    """``count`` matrix orders log-uniform in [n_min, n_max]:
    n = round(exp(U(ln n_min, ln n_max)))."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(n_min), math.log(n_max), size=count)
    return [int(min(n_max, max(n_min, round(math.exp(x))))) for x in u]


def _perm_sign(perm: np.ndarray) -> int:
    """Sign of a permutation, by counting cycles (sign = (-1)^(n - #cycles))."""
    n = len(perm)
    seen = np.zeros(n, dtype=bool)
    cycles = 0
    for i in range(n):
        if not seen[i]:
            cycles += 1
            j = i
            while not seen[j]:
                seen[j] = True
                j = int(perm[j])
    return -1 if (n - cycles) % 2 else 1


def _unit_triangular(n: int, rng: np.random.Generator, lower: bool, density: float) -> np.ndarray:
    """Unit triangular integer matrix; each off-diagonal entry of the
    triangle is +1 or -1 with probability ``density`` (equally likely), else 0."""
    t = np.eye(n, dtype=np.int64)
    mask = rng.random((n, n)) < density
    signs = np.where(rng.random((n, n)) < 0.5, -1, 1).astype(np.int64)
    tri = np.tril(np.ones((n, n), dtype=bool), -1) if lower else np.triu(np.ones((n, n), dtype=bool), 1)
    t[mask & tri] = signs[mask & tri]
    return t


def _matmul_exact(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Exact int64 product for sparse-ish integer factors (checked against
    overflow through a float64 bound on |a| |b|)."""
    bound = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
    if bound.size and bound.max() >= 2.0 ** 62:
        raise OverflowError("integer product would overflow int64")
    import scipy.sparse as sp

    return np.asarray((sp.csr_matrix(a) @ sp.csr_matrix(b)).toarray(), dtype=np.int64)


def unimodular_factors(n: int, seed: int, density: float | None = None):
    """Random unimodular U = P1 L1 R1 and V = L2 R2 P2 (P permutation, L unit
    lower, R unit upper triangular).  Returns (U, V, sign) with
    sign = det(U) * det(V) = sign(P1) * sign(P2), known by construction."""
    rng = np.random.default_rng(seed)
    if density is None:
        density = min(1.0, 3.0 / max(n, 1))
    p1 = rng.permutation(n)
    p2 = rng.permutation(n)
    l1 = _unit_triangular(n, rng, True, density)
    r1 = _unit_triangular(n, rng, False, density)
    l2 = _unit_triangular(n, rng, True, density)
    r2 = _unit_triangular(n, rng, False, density)
    P1 = np.zeros((n, n), dtype=np.int64)
    P1[np.arange(n), p1] = 1
    P2 = np.zeros((n, n), dtype=np.int64)
    P2[np.arange(n), p2] = 1
    U = _matmul_exact(P1, _matmul_exact(l1, r1))
    V = _matmul_exact(_matmul_exact(l2, r2), P2)
    return U, V, _perm_sign(p1) * _perm_sign(p2)


def smith_matrix(s, seed: int, density: float | None = None):
    """A = U diag(s) V with random unimodular U, V.  Returns (A, sign) where
    det(A) = sign * prod(s).  The invariant factors of A are those of
    diag(s) (unimodular equivalence preserves the Smith form)."""
    s = np.asarray([int(v) for v in s], dtype=np.int64)
    n = len(s)
    U, V, sign = unimodular_factors(n, seed, density)
    A = _matmul_exact(U * s[np.newaxis, :], V)
    return A, sign


def engineered_table1(n: int, seed: int, density: float | None = None):
    """Matrix with the Smith form of diag(1, 2, ..., n) (the Table 1
    workload): det = sign * n!, largest invariant factor lcm(1..n)."""
    return smith_matrix(range(1, n + 1), seed, density)


def structured_serving(n: int, seed: int):
    """Invariant factors (1,..,1, s_{n-m+1},..,s_n) with m ~ U{2..5},
    s_{n-m+1} ~ U{2..9} and each next factor the previous times U{2..9}.
    Returns (A, sign, s) with det(A) = sign * prod(s)."""
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 6))
    tail = [int(rng.integers(2, 10))]
    for _ in range(m - 1):
        tail.append(tail[-1] * int(rng.integers(2, 10)))
    s = [1] * (n - m) + tail
    A, sign = smith_matrix(s, seed + 0x5EED, None)
    return A, sign, s


def random_rhs(n: int, beta: int, seed: int) -> np.ndarray:
    """Right-hand side b with entries uniform in [0, beta)."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, beta, size=n, dtype=np.int64)


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson stream: cumulative exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))
