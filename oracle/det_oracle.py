"""Plain, slow, obviously correct reference computations (test infrastructure
only; see the package docstring).  Integers are Python ``int`` unless a numpy
int64 bound is checked first.

Paper: J.-G. Dumas and A. Urbanska, "An introspective algorithm for the
integer determinant".  Section numbers below refer to it.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


# --------------------------------------------------------------------------
# O1: det(A) by the textbook definition, via fraction-free elimination.
# --------------------------------------------------------------------------
def det_bareiss(A) -> int:
    """Exact det(A) by Bareiss fraction-free elimination over Python ints.

    The paper relies on det(A) itself (Section 2.1 reconstructs it); this is
    the textbook exact algorithm: after step k every entry below/right of the
    pivot is a (k+1)x(k+1) minor, so division by the previous pivot is exact.
    A zero pivot is replaced by the first lower row with a non-zero entry in
    that column (one row swap, sign flip); no such row means det = 0.
    n = 0 gives 1 (empty product)."""
    M = [[int(x) for x in row] for row in np.asarray(A, dtype=object).tolist()] if len(A) else []
    n = len(M)
    if n == 0:
        return 1
    sign = 1
    prev = 1
    for k in range(n - 1):
        if M[k][k] == 0:
            for i in range(k + 1, n):
                if M[i][k] != 0:
                    M[k], M[i] = M[i], M[k]
                    sign = -sign
                    break
            else:
                return 0
        akk = M[k][k]
        rowk = M[k]
        for i in range(k + 1, n):
            rowi = M[i]
            aik = rowi[k]
            for j in range(k + 1, n):
                q, r = divmod(akk * rowi[j] - aik * rowk[j], prev)
                assert r == 0, "Bareiss division must be exact"
                rowi[j] = q
            rowi[k] = 0
        prev = akk
    return sign * M[n - 1][n - 1]


# --------------------------------------------------------------------------
# O2: det(A) mod p by Gaussian elimination over Z_p.
# --------------------------------------------------------------------------
def _check_modulus(p: int) -> None:
    if p < 2 or p >= 1 << 31:
        raise ValueError("modulus out of the int64-safe range")


def det_mod_p(A, p: int) -> int:
    """det(A) mod p in [0, p) by LU over Z_p (Section 2.1 computes each
    modular determinant by an LU factorisation modulo p_i).

    Pivot: the first row at or below the diagonal whose entry is non-zero
    mod p; each swap flips the sign.  det = sign * prod(pivots) mod p.  A
    column without pivot means det = 0 mod p.  Every product is reduced at
    once (entries < p < 2^31, so products < 2^62 fit int64)."""
    _check_modulus(p)
    M = np.asarray(A, dtype=np.int64) % p
    n = M.shape[0]
    det = 1
    for k in range(n):
        nz = np.nonzero(M[k:, k])[0]
        if len(nz) == 0:
            return 0
        piv = k + int(nz[0])
        if piv != k:
            M[[k, piv]] = M[[piv, k]]
            det = -det
        pk = int(M[k, k])
        det = det * pk % p
        inv = pow(pk, -1, p)
        f = (M[k + 1:, k] * inv) % p
        # each product f_i * u_kj < p^2 < 2^62: no int64 overflow
        M[k + 1:, k + 1:] = (M[k + 1:, k + 1:] - np.outer(f, M[k, k + 1:]) % p) % p
    return det % p


def inverse_mod_p(A, p: int) -> np.ndarray:
    """A^{-1} mod p (entries in [0, p)) by Gauss-Jordan over Z_p on [A | I].
    Raises ZeroDivisionError if p divides det(A)."""
    _check_modulus(p)
    A = np.asarray(A, dtype=np.int64) % p
    n = A.shape[0]
    M = np.concatenate([A, np.eye(n, dtype=np.int64)], axis=1)
    for k in range(n):
        nz = np.nonzero(M[k:, k])[0]
        if len(nz) == 0:
            raise ZeroDivisionError("A is singular modulo p")
        piv = k + int(nz[0])
        if piv != k:
            M[[k, piv]] = M[[piv, k]]
        inv = pow(int(M[k, k]), -1, p)
        M[k] = (M[k] * inv) % p
        f = M[:, k].copy()
        f[k] = 0
        # eliminate column k from every other row; products < p^2 < 2^62
        M = (M - np.outer(f, M[k]) % p) % p
    return M[:, n:].copy()


# --------------------------------------------------------------------------
# O3: Dixon p-adic digits (Section 2.2, the solver of LargestInvariantFactor).
# --------------------------------------------------------------------------
def _matvec_mod(C: np.ndarray, v: np.ndarray, p: int) -> np.ndarray:
    """C v mod p with C, v in [0, p): row sums taken over column chunks small
    enough that no int64 partial sum can overflow."""
    n = C.shape[1]
    chunk = max(1, (1 << 62) // max(1, (p - 1) * (p - 1)))
    out = np.zeros(C.shape[0], dtype=np.int64)
    for c0 in range(0, n, chunk):
        out = (out + (C[:, c0:c0 + chunk] @ v[c0:c0 + chunk]) % p) % p
    return out


def dixon_digits(A, b, p: int, k: int) -> np.ndarray:
    """The first k base-p digit vectors x_0..x_{k-1} of x = A^{-1} b in Z_p.

    Dixon lifting: r_0 = b; x_i is the unique vector in [0,p)^n with
    A x_i = r_i (mod p); r_{i+1} = (r_i - A x_i)/p, an exact division.
    Then sum_i x_i p^i = A^{-1} b (mod p^k).  Returns a k x n int64 array.
    The residual update runs in int64 when n ||A|| p + ||b|| < 2^62 (then no
    intermediate can overflow) and on Python ints otherwise."""
    A = np.asarray(A, dtype=np.int64)
    n = A.shape[0]
    C = inverse_mod_p(A, p)
    digits = np.zeros((k, n), dtype=np.int64)
    amax = int(np.abs(A).max()) if A.size else 0
    bmax = max([abs(int(v)) for v in b] + [0])
    # |r_i| <= max(|b|, n ||A|| p): int64 is exact if that and |A x| stay
    # far below 2^63; otherwise fall back to Python ints.
    small = n * amax * p + bmax < (1 << 62)
    if small:
        r = np.asarray([int(v) for v in b], dtype=np.int64)
        Aw = A
    else:
        r = np.asarray([int(v) for v in b], dtype=object)
        Aw = A.astype(object)
    for i in range(k):
        rp = np.asarray([int(v) % p for v in r], dtype=np.int64)
        x = _matvec_mod(C, rp, p)
        digits[i] = x
        t = r - Aw.dot(x if small else x.astype(object))
        if any(int(v) % p for v in t):
            raise AssertionError("residual must be divisible by p")
        r = t // p
    return digits


# --------------------------------------------------------------------------
# O7: Hadamard bound (Lemma 2.1 uses H = (sqrt(n) ||A||)^n; the column and
# row norm forms are tighter bounds of the same inequality).
# --------------------------------------------------------------------------
def hadamard_sq(A) -> int:
    """min(prod_j ||a_j||^2 over columns, prod_i ||a^i||^2 over rows) as an
    exact integer: |det A|^2 <= this value (Hadamard's inequality)."""
    M = [[int(x) for x in row] for row in np.asarray(A, dtype=object).tolist()]
    n = len(M)
    if n == 0:
        return 1
    rows = 1
    for row in M:
        rows *= sum(x * x for x in row)
    cols = 1
    for j in range(n):
        cols *= sum(M[i][j] * M[i][j] for i in range(n))
    return min(rows, cols)


def hadamard_bits(A) -> int:
    """Smallest integer b with 2^b >= sqrt(hadamard_sq(A)), i.e. an exact,
    upward-rounded log2 of the Hadamard bound (0 when the bound is <= 1)."""
    h2 = hadamard_sq(A)
    if h2 <= 1:
        return 0
    two_b = (h2 - 1).bit_length()      # smallest e with 2^e >= h2
    return (two_b + 1) // 2            # smallest b with 2^(2b) >= h2


# --------------------------------------------------------------------------
# O4: exact rational solution and the denominator that LIF returns.
# --------------------------------------------------------------------------
def solve_rational(A, b):
    """x = A^{-1} b over Q by Gaussian elimination with Python Fractions.
    Returns (num, den): integer vector num and den > 0, with x = num/den and
    den the least common denominator of the entries of x (Section 2.2:
    d(x), which divides s_n)."""
    n = len(A)
    M = [[Fraction(int(v)) for v in row] + [Fraction(int(bi))]
         for row, bi in zip(np.asarray(A, dtype=object).tolist(), list(b))]
    for k in range(n):
        piv = next((i for i in range(k, n) if M[i][k] != 0), None)
        if piv is None:
            raise ZeroDivisionError("A is singular")
        M[k], M[piv] = M[piv], M[k]
        for i in range(k + 1, n):
            if M[i][k] != 0:
                f = M[i][k] / M[k][k]
                M[i] = [a - f * c for a, c in zip(M[i], M[k])]
    x = [Fraction(0)] * n
    for k in range(n - 1, -1, -1):
        s = M[k][n] - sum(M[k][j] * x[j] for j in range(k + 1, n))
        x[k] = s / M[k][k]
    den = 1
    for v in x:
        den = den * v.denominator // math.gcd(den, v.denominator)
    num = [int(v * den) for v in x]
    return num, den


def largest_invariant_factor(A, bs) -> int:
    """s~_n = lcm over the right-hand sides b of d(A^{-1} b) (Section 2.2:
    each solving updates s~_n as the lcm of the current denominator and the
    result so far)."""
    s = 1
    for b in bs:
        _, d = solve_rational(A, b)
        s = s * d // math.gcd(s, d)
    return s


def extended_bonus(A, B, R):
    """pi~ of the extended bonus (Section 3.2, "the last k invariant factors";
    Alg. 4.1 with i right-hand sides): the columns b_1..b_i of B solved over
    Q, s~ = lcm of their common denominators (Section 2.2), N = s~ X with
    X = [x_1..x_i], and for the random i x n matrix R
        pi~ = s~^i / gcd(det(R N), s~^i),
    a factor of s_n s_{n-1} ... s_{n-i+1} (equal to it with high probability).
    Returns (s~, pi~)."""
    B = [[int(v) for v in row] for row in np.asarray(B, dtype=object).tolist()]
    i = len(B[0])
    sols = [solve_rational(A, [row[h] for row in B]) for h in range(i)]
    s = 1
    for _, d in sols:
        s = s * d // math.gcd(s, d)
    # N = s~ X: column h is num_h * (s~ / d_h)
    N = [[num[j] * (s // d) for num, d in sols] for j in range(len(A))]
    R = [[int(v) for v in row] for row in np.asarray(R, dtype=object).tolist()]
    RN = [[sum(R[a][j] * N[j][h] for j in range(len(A))) for h in range(i)] for a in range(i)]
    dRN = det_bareiss(RN) if i > 0 else 1
    si = s ** i
    return s, si // math.gcd(dRN, si)


def dixon_length(A, b, p: int) -> int:
    """Smallest k with p^k > 2 N D, where D = H (Hadamard) bounds the common
    denominator and N = H ||b|| / min_j ||a_j|| bounds every Cramer numerator
    det(A_j) (A_j = A with column j replaced by b).  Squared, exactly:
    p^(2k) * min_j ||a_j||^2 > 4 * H^4 * ||b||^2 with H^2 the column form."""
    M = np.asarray(A, dtype=object)
    n = M.shape[0]
    col_sq = [sum(int(M[i, j]) ** 2 for i in range(n)) for j in range(n)]
    h2 = 1
    for c in col_sq:
        h2 *= c
    b2 = sum(int(v) ** 2 for v in b)
    rhs = 4 * h2 * h2 * max(b2, 1)
    cmin = max(1, min(col_sq))
    k = 0
    while p ** (2 * k) * cmin <= rhs:
        k += 1
    return k


# --------------------------------------------------------------------------
# O5: Chinese remaindering in the symmetric range, and early termination.
# --------------------------------------------------------------------------
def crt_symmetric(residues, primes) -> tuple[int, int]:
    """The unique r with r = d_i (mod p_i) for all i and
    -floor(M/2) <= r < ceil(M/2), M = prod p_i (Section 2.1, proof of
    Lemma 2.1(i)).  Plain formula r = sum d_i (M/p_i) ((M/p_i)^{-1} mod p_i).
    Returns (r, M)."""
    M = 1
    for p in primes:
        M *= int(p)
    r = 0
    for d, p in zip(residues, primes):
        p = int(p)
        Mi = M // p
        r += int(d) * Mi * pow(Mi % p, -1, p)
    r %= M
    if r >= (M + 1) // 2:      # ceil(M/2) <= r  ->  shift into the range
        r -= M
    return r, M


def et_k(log2_inv_eps: float, P_size: int, logl_H: int) -> int:
    """Number of unchanged reconstructions that Lemma 2.1(iv) requires:
    k = ceil(log(1/eps) / (log P' - log log_l H)), P' = |P| - ceil(log_l H)."""
    Pp = P_size - logl_H
    denom = math.log2(Pp) - math.log2(max(logl_H, 1))
    if denom <= 0:
        raise ValueError("prime set too small for early termination")
    return max(1, math.ceil(log2_inv_eps / denom))


def et_cra(residues, primes, H_bits: int, k: int):
    """Early-terminated CRA (Alg. 2.1) read with the closed form of Lemma
    2.1(iv): process (d_i, p_i) in the given order, reconstruct r_i in the
    symmetric range, stop once r stayed the same for k consecutive new
    primes, or deterministically once prod p_i >= 2 H (H = 2^H_bits).
    "Unchanged" means r_{i-1} = d_i (mod p_i), which is exactly r_i = r_{i-1}.
    Returns (r, primes_used, early) or None when the list runs out first."""
    r = None
    M = 1
    same = 0
    used_d, used_p = [], []
    for d, p in zip(residues, primes):
        p = int(p)
        d = int(d) % p
        if r is not None and (r - d) % p == 0:
            same += 1
        else:
            same = 0
        used_d.append(d)
        used_p.append(p)
        r, M = crt_symmetric(used_d, used_p)
        if M >= 2 * (1 << H_bits):
            return r, len(used_p), False
        if same >= k:
            return r, len(used_p), True
    return None


# --------------------------------------------------------------------------
# O6: rational number reconstruction.
# --------------------------------------------------------------------------
def rational_reconstruct(u: int, m: int, N: int, D: int):
    """Find a/d with a = u d (mod m), |a| <= N, 0 < d <= D, gcd(a, d) = 1.
    Unique when 2 N D < m.  Extended Euclid on (m, u mod m), stopped at the
    first remainder <= N (Wang's method).  Returns (a, d) or None."""
    u %= m
    r0, r1 = m, u
    t0, t1 = 0, 1
    while r1 > N:
        q = r0 // r1
        r0, r1 = r1, r0 - q * r1
        t0, t1 = t1, t0 - q * t1
    a, d = r1, t1
    if d == 0:
        return None
    if d < 0:
        a, d = -a, -d
    if d > D or math.gcd(a, d) != 1:
        return None
    if (a - u * d) % m != 0:
        return None
    return a, d


# --------------------------------------------------------------------------
# Small helpers used by the tests.
# --------------------------------------------------------------------------
def is_prime(q: int) -> bool:
    """Trial division (plain definition), fine for q < 2^32."""
    if q < 2:
        return False
    if q % 2 == 0:
        return q == 2
    f = 3
    while f * f <= q:
        if q % f == 0:
            return False
        f += 2
    return True


def det_introspective_oracle(A) -> int:
    """The exact value that the introspective algorithm returns (its
    certified result is det(A) itself): det_bareiss."""
    return det_bareiss(A)
