"""Pins for the CPU oracle, against what the paper and the mathematics fix
(never against the oracle itself).  CPU only.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, an off-by-one bound) fails it.
"""
import itertools
import math
import random

import numpy as np
import pytest

import oracle
import synth
from conftest import test_primes


# ---------------------------------------------------------------- helpers
def det_cofactor(M):
    """Laplace expansion along the first row (brute force, n <= 8)."""
    M = [list(map(int, r)) for r in M]
    n = len(M)
    if n == 0:
        return 1
    if n == 1:
        return M[0][0]
    total = 0
    for j in range(n):
        if M[0][j] == 0:
            continue
        minor = [row[:j] + row[j + 1:] for row in M[1:]]
        total += (-1) ** j * M[0][j] * det_cofactor(minor)
    return total


def det_leibniz(M):
    """Sum over permutations (n <= 6), an independent second definition."""
    n = len(M)
    total = 0
    for perm in itertools.permutations(range(n)):
        inv = sum(1 for i in range(n) for j in range(i + 1, n) if perm[i] > perm[j])
        prod = 1
        for i in range(n):
            prod *= int(M[i][perm[i]])
        total += (-1) ** inv * prod
    return total


def matmul_int(A, B):
    A = [list(map(int, r)) for r in A]
    B = [list(map(int, r)) for r in B]
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


# ---------------------------------------------------------------- O1 pins
@pytest.mark.parametrize("n", range(0, 8))
def test_bareiss_equals_cofactor_expansion(n):
    for seed in range(4):
        A = synth.dense_uniform(n, -9, 9, 100 * n + seed)
        assert oracle.det_bareiss(A) == det_cofactor(A)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_bareiss_equals_leibniz(n):
    A = synth.dense_uniform(n, -100, 100, 7 + n)
    assert oracle.det_bareiss(A) == det_leibniz(A)


def test_bareiss_triangular_is_diagonal_product():
    rng = np.random.default_rng(3)
    for n in (1, 5, 17, 40):
        T = np.triu(rng.integers(-50, 51, size=(n, n)))
        d = [int(v) for v in rng.integers(1, 30, size=n) * rng.choice([-1, 1], size=n)]
        np.fill_diagonal(T, d)
        assert oracle.det_bareiss(T) == math.prod(d)
        assert oracle.det_bareiss(T.T.copy()) == math.prod(d)


def test_bareiss_multiplicative():
    for n, seed in ((6, 1), (20, 2)):
        A = synth.dense_uniform(n, -20, 20, seed)
        B = synth.dense_uniform(n, -20, 20, seed + 50)
        AB = matmul_int(A, B)
        assert oracle.det_bareiss(AB) == oracle.det_bareiss(A) * oracle.det_bareiss(B)


def test_bareiss_row_swap_flips_sign():
    A = synth.dense_uniform(12, -100, 100, 11)
    B = A.copy()
    B[[2, 9]] = B[[9, 2]]
    d = oracle.det_bareiss(A)
    assert d != 0 and oracle.det_bareiss(B) == -d
    C = A.copy()
    C[:, [0, 5]] = C[:, [5, 0]]
    assert oracle.det_bareiss(C) == -d


def test_bareiss_zero_pivot_and_singular():
    A = synth.dense_uniform(7, -5, 5, 4)
    A[0, 0] = 0
    A[1, 0] = 0
    assert oracle.det_bareiss(A) == det_cofactor(A)
    S = A.copy()
    S[4] = 2 * S[1] - 3 * S[6]          # rank deficient
    assert oracle.det_bareiss(S) == 0
    Z = np.zeros((5, 5), dtype=np.int64)
    assert oracle.det_bareiss(Z) == 0
    E = np.zeros((3, 3), dtype=np.int64)
    E[0, 2] = E[1, 1] = E[2, 0] = 1     # anti-diagonal: one swap, det = -1
    assert oracle.det_bareiss(E) == -1


@pytest.mark.parametrize("n", [8, 24, 60])
def test_bareiss_smith_construction(n):
    """det(U diag(s) V) = +-prod(s) with the sign fixed by the permutations."""
    rng = np.random.default_rng(n)
    s = sorted(int(v) for v in rng.integers(1, 12, size=n))
    A, sign = synth.smith_matrix(s, seed=n + 1, density=0.3)
    assert oracle.det_bareiss(A) == sign * math.prod(s)


def test_table1_engineered_det_is_factorial():
    """Table 1 matrices have the Smith form of diag(1..n): det = +-n!."""
    for n in (10, 40):
        A, sign = synth.engineered_table1(n, seed=n)
        assert oracle.det_bareiss(A) == sign * math.factorial(n)


def test_hadamard_bound_holds():
    """|det A| <= prod_j ||a_j|| (Lemma 2.1 uses the cruder (sqrt(n)||A||)^n)."""
    for n, lo, hi, seed in ((16, -100, 100, 1), (40, 0, 255, 2), (30, -1024, 1024, 3)):
        A = synth.dense_uniform(n, lo, hi, seed)
        d = oracle.det_bareiss(A)
        h2 = oracle.hadamard_sq(A)
        assert d * d <= h2
        bits = oracle.hadamard_bits(A)
        assert (1 << (2 * bits)) >= h2 > (1 << (2 * (bits - 1)))
        amax = int(np.abs(A).max())
        assert h2 <= (n * amax * amax) ** n       # crude bound of the paper
    # an orthogonal matrix meets the bound with equality
    Hm = np.array([[1, 1, 1, 1], [1, -1, 1, -1], [1, 1, -1, -1], [1, -1, -1, 1]])
    assert oracle.hadamard_sq(Hm) == oracle.det_bareiss(Hm) ** 2 == 256
    assert oracle.hadamard_bits(Hm) == 4


@pytest.mark.parametrize("n", [12, 32])
def test_bareiss_matches_sympy(n):
    sympy = pytest.importorskip("sympy")
    A = synth.dense_uniform(n, -100, 100, 1000 + n)
    assert oracle.det_bareiss(A) == int(sympy.Matrix(A.tolist()).det(method="bareiss"))


@pytest.mark.parametrize("n", [0, 1, 2, 9, 33, 70])
def test_c_bareiss_matches_python_bareiss(n):
    for lo, hi in ((-100, 100), (0, 255)):
        A = synth.dense_uniform(n, lo, hi, n + hi)
        assert oracle.det_bareiss_c(A) == oracle.det_bareiss(A)


def test_c_bareiss_special_cases():
    A = synth.dense_uniform(20, -3, 3, 5)
    A[:, 0] = 0
    A[7, 0] = 2                          # forces a swap at k = 0
    assert oracle.det_bareiss_c(A) == oracle.det_bareiss(A)
    S = A.copy()
    S[3] = S[5] + S[8]
    assert oracle.det_bareiss_c(S) == 0
    big = synth.dense_uniform(6, -(2 ** 40), 2 ** 40, 9)     # multi-limb entries
    assert oracle.det_bareiss_c(big) == det_cofactor(big)
    A, sign = synth.engineered_table1(48, seed=3)
    assert oracle.det_bareiss_c(A) == sign * math.factorial(48)


# ---------------------------------------------------------------- O2 pins
def test_det_mod_p_matches_exact_det():
    for n, seed in ((1, 1), (5, 2), (33, 3), (64, 4)):
        A = synth.dense_uniform(n, -100, 100, seed)
        d = oracle.det_bareiss(A)
        for p in test_primes(1 << 22, 1 << 23, 3, seed) + test_primes(1 << 25, 1 << 26, 2, seed) + [3, 5]:
            assert oracle.det_mod_p(A, p) == d % p


def test_det_mod_p_prime_divides_det_and_singular():
    p = test_primes(1 << 22, 1 << 23, 1, 77)[0]
    s = [1] * 20 + [p]
    A, _ = synth.smith_matrix(s, seed=5, density=0.3)
    assert oracle.det_mod_p(A, p) == 0
    q = test_primes(1 << 22, 1 << 23, 1, 78)[0]
    assert oracle.det_mod_p(A, q) == oracle.det_bareiss(A) % q != 0
    S = synth.dense_uniform(16, -50, 50, 6)
    S[10] = S[2] - S[3]
    for q in test_primes(1 << 20, 1 << 26, 4, 79):
        assert oracle.det_mod_p(S, q) == 0


def test_inverse_mod_p_is_an_inverse():
    A = synth.dense_uniform(40, -100, 100, 21)
    for p in test_primes(1 << 22, 1 << 23, 2, 21):
        C = oracle.inverse_mod_p(A, p)
        AC = (np.asarray(matmul_int(A, C), dtype=object) % p).astype(np.int64)
        assert np.array_equal(AC, np.eye(40, dtype=np.int64))
        assert C.min() >= 0 and C.max() < p


# ---------------------------------------------------------------- O3/O4 pins
def test_solve_rational_satisfies_system():
    for n, seed in ((1, 1), (6, 2), (25, 3)):
        A = synth.dense_uniform(n, -100, 100, seed)
        b = synth.random_rhs(n, 1000, seed)
        num, den = oracle.solve_rational(A, b)
        assert den > 0
        Anum = matmul_int(A, [[v] for v in num])
        assert [r[0] for r in Anum] == [den * int(v) for v in b]
        assert math.gcd(den, *num) == 1 or all(v == 0 for v in num)
        assert oracle.det_bareiss(A) % den == 0            # d(x) | s_n | det


def test_solve_rational_matches_cramer():
    """x_j = det(A_j)/det(A), with A_j = A with column j replaced by b."""
    A = synth.dense_uniform(5, -9, 9, 31)
    b = synth.random_rhs(5, 50, 31)
    num, den = oracle.solve_rational(A, b)
    d = det_cofactor(A)
    for j in range(5):
        Aj = A.copy()
        Aj[:, j] = b
        assert num[j] * d == det_cofactor(Aj) * den


def test_lif_denominator_divides_largest_invariant_factor():
    """Section 2.2: d(x) | s_n.  With A = U diag(s) V, s_n is known."""
    s = [1] * 12 + [2, 6, 30]
    A, _ = synth.smith_matrix(s, seed=4, density=0.4)
    hits = 0
    for seed in range(8):
        b = synth.random_rhs(len(s), 1000, seed)
        _, den = oracle.solve_rational(A, b)
        assert 30 % den == 0
        hits += den == 30
    assert hits >= 2      # Thm 2.2(i): each prime power is missed with prob ~1/p^l


def test_table1_lif_two_solves():
    """Table 1 matrices: s_n = lcm(1..n); two solves (r = 2) with
    beta = 6 + 2 ceil(log2 H) give s_n with probability >= 1/3 (Thm 2.2(iii))."""
    n = 14
    A, _ = synth.engineered_table1(n, seed=2)
    sn = math.lcm(*range(1, n + 1))
    beta = 6 + 2 * oracle.hadamard_bits(A)
    hits = 0
    for t in range(6):
        bs = [synth.random_rhs(n, beta, 100 + 2 * t), synth.random_rhs(n, beta, 101 + 2 * t)]
        s = oracle.largest_invariant_factor(A, bs)
        assert sn % s == 0
        hits += s == sn
    assert hits >= 1


def test_dixon_digits_invariants():
    """Checked without the inverse: A x_i = r_i (mod p), p | r_i - A x_i,
    and sum x_i p^i = num * den^{-1} (mod p^k) from the exact solution."""
    n = 20
    A = synth.dense_uniform(n, -100, 100, 8)
    b = synth.random_rhs(n, 500, 8)
    p = test_primes(1 << 22, 1 << 23, 1, 8)[0]
    k = 12
    X = oracle.dixon_digits(A, b, p, k)
    assert X.shape == (k, n) and X.min() >= 0 and X.max() < p
    r = [int(v) for v in b]
    for i in range(k):
        Ax = [sum(int(A[a, c]) * int(X[i, c]) for c in range(n)) for a in range(n)]
        t = [r[a] - Ax[a] for a in range(n)]
        assert all(v % p == 0 for v in t)
        r = [v // p for v in t]
    num, den = oracle.solve_rational(A, b)
    pk = p ** k
    inv = pow(den, -1, pk)
    for j in range(n):
        val = sum(int(X[i, j]) * p ** i for i in range(k))
        assert val == num[j] * inv % pk


def test_dixon_length_bound():
    A = synth.dense_uniform(10, -100, 100, 3)
    b = synth.random_rhs(10, 100, 3)
    p = 1000003
    k = oracle.dixon_length(A, b, p)
    num, den = oracle.solve_rational(A, b)
    N = max(abs(v) for v in num)
    assert p ** k > 2 * N * den
    # the digits reconstruct x: rational reconstruction recovers every entry
    X = oracle.dixon_digits(A, b, p, k)
    pk = p ** k
    for j in range(10):
        u = sum(int(X[i, j]) * p ** i for i in range(k))
        a, d = oracle.rational_reconstruct(u, pk, (pk - 1) // (2 * den), den)
        from fractions import Fraction
        assert Fraction(a, d) == Fraction(num[j], den)


# ---------------------------------------------------------------- O5 pins
def test_crt_symmetric_range_and_sympy():
    from sympy.ntheory.modular import crt
    ps = test_primes(1 << 22, 1 << 23, 5, 12)
    rng = random.Random(5)
    for _ in range(20):
        ds = [rng.randrange(p) for p in ps]
        r, M = oracle.crt_symmetric(ds, ps)
        assert M == math.prod(ps)
        assert -(M // 2) <= r < (M + 1) // 2
        assert all((r - d) % p == 0 for d, p in zip(ds, ps))
        assert r % M == int(crt(ps, ds)[0])


def test_crt_recovers_det_once_product_exceeds_twice_det():
    """Lemma 2.1(i): r_t = det(A) as soon as prod p >= 2 |det A|."""
    A = synth.dense_uniform(30, -100, 100, 13)
    d = oracle.det_bareiss(A)
    ps = test_primes(1 << 22, 1 << 23, 40, 13)
    used = []
    for p in ps:
        used.append(p)
        r, M = oracle.crt_symmetric([d % q for q in used], used)
        if M >= 2 * abs(d):
            assert r == d
            break
    else:
        pytest.fail("not enough primes")
    assert oracle.crt_symmetric([0, 0, 0], ps[:3])[0] == 0
    assert oracle.crt_symmetric([p - 1 for p in ps[:3]], ps[:3])[0] == -1


def test_et_k_is_minimal_for_the_lemma_bound():
    """Lemma 2.1(iv): the smallest k with (log_l H / P')^k < eps."""
    for eps_bits, P, L in ((64, 268000, 568), (20, 5000, 30), (64, 3000, 900)):
        k = oracle.et_k(eps_bits, P, L)
        ratio = L / (P - L)
        assert ratio ** k <= 2.0 ** -eps_bits * (1 + 1e-9)
        if k > 1:
            assert ratio ** (k - 1) > 2.0 ** -eps_bits
    with pytest.raises(ValueError):
        oracle.et_k(64, 1000, 900)       # |P| too small for the lemma


def test_et_cra_returns_det():
    for n, seed in ((12, 1), (40, 2)):
        A = synth.dense_uniform(n, -100, 100, seed)
        d = oracle.det_bareiss(A)
        hb = oracle.hadamard_bits(A)
        ps = test_primes(1 << 22, 1 << 23, hb // 22 + 12, seed)
        res = [oracle.det_mod_p(A, p) for p in ps]
        r, used, early = oracle.et_cra(res, ps, hb, k=3)
        assert r == d
        # a huge k forces the deterministic Hadamard stop
        r2, used2, early2 = oracle.et_cra(res, ps, hb, k=10 ** 6)
        assert r2 == d and not early2 and math.prod(ps[:used2]) >= 2 << hb
        assert math.prod(ps[:used2 - 1]) < 2 << hb
    # det = 0: all residues 0, ET after k + 1 primes
    r, used, early = oracle.et_cra([0] * 10, ps[:10], 500, k=3)
    assert (r, used, early) == (0, 4, True)


def test_et_cra_counts_only_consecutive_agreement():
    ps = test_primes(1 << 22, 1 << 23, 8, 99)
    target = -1234567
    res = [target % p for p in ps]
    assert oracle.et_cra(res, ps, 2000, k=2) == (target, 3, True)
    assert oracle.et_cra(res, ps, 2000, k=5) == (target, 6, True)
    bad = list(res)
    bad[1] = (bad[1] + 1) % ps[1]       # a wrong residue breaks the run for good
    assert oracle.et_cra(bad, ps, 2000, k=2) is None


# ---------------------------------------------------------------- O6 pins
def test_rational_reconstruction_recovers_fraction():
    rng = random.Random(17)
    m = (1 << 127) - 1
    for _ in range(200):
        d = rng.randrange(1, 1 << 60)
        a = rng.randrange(-(1 << 60), 1 << 60)
        g = math.gcd(a, d)
        a, d = a // g, d // g
        u = a * pow(d, -1, m) % m
        N = D = 1 << 60
        assert 2 * N * D < m
        assert oracle.rational_reconstruct(u, m, N, D) == (a, d)
    assert oracle.rational_reconstruct(5, 101, 7, 7) == (5, 1)
    assert oracle.rational_reconstruct(0, 101, 7, 7) == (0, 1)


def test_rational_reconstruction_rejects_out_of_bounds():
    m = 10007
    u = 1234 * pow(5678, -1, m) % m
    out = oracle.rational_reconstruct(u, m, 70, 70)
    assert out is None or (abs(out[0]) <= 70 and 0 < out[1] <= 70 and (out[0] - u * out[1]) % m == 0)


def test_is_prime_trial_division():
    sympy = pytest.importorskip("sympy")
    for q in list(range(0, 2000)) + [2 ** 23 - 15, 2 ** 25 + 35, 2 ** 26 - 5]:
        assert oracle.is_prime(q) == bool(sympy.isprime(q))


# ---------------------------------------------------------------- planted mistakes
def _pins_hold(det) -> bool:
    """The determinant pins of this file, run against a candidate `det`:
    cofactor expansion (matrices with zero leading entries, so row swaps
    happen), triangular products, det(AB) = det(A) det(B), a row swap flips
    the sign, and Smith-form constructions with a known determinant."""
    try:
        rng = np.random.default_rng(2024)
        for n in (3, 4, 5, 6):
            for _ in range(4):
                A = rng.integers(-9, 10, size=(n, n))
                A[0, 0] = 0
                if det(A) != det_cofactor(A):
                    return False
        T = np.triu(rng.integers(-9, 10, size=(7, 7)))
        if det(T) != int(np.prod([int(v) for v in np.diag(T)])):
            return False
        A = rng.integers(-5, 6, size=(6, 6))
        B = rng.integers(-5, 6, size=(6, 6))
        if det(A @ B) != det(A) * det(B):
            return False
        S = A.copy()
        S[[1, 4]] = S[[4, 1]]
        if det(S) != -det(A):
            return False
        M, sign = synth.smith_matrix([1, 1, 2, 6, 30], 5, 0.5)
        if det(M) != sign * 360:
            return False
    except Exception:          # a planted slip may also break the exact division
        return False
    return True


# each mutation is one plausible slip in the elimination: a dropped sign
# flip, a transposed operand, a wrong pivot divisor, an off-by-one index, a
# lost pivot search
_MUTATIONS = [
    ("sign = -sign", "sign = sign"),
    ("akk * rowi[j] - aik * rowk[j]", "aik * rowk[j] - akk * rowi[j]"),
    ("prev = akk", "prev = 1"),
    ("aik * rowk[j]", "aik * rowk[j - 1]"),
    ("return sign * M[n - 1][n - 1]", "return sign * M[n - 1][n - 2]"),
    ("if M[k][k] == 0:", "if False:"),
]


@pytest.mark.parametrize("old,new", _MUTATIONS)
def test_pins_catch_a_planted_mistake(old, new):
    """A slip planted into a copy of the oracle's Bareiss elimination fails
    the pins, while the oracle itself passes them."""
    import inspect
    import textwrap

    from oracle import det_oracle as m

    assert _pins_hold(m.det_bareiss)
    src = textwrap.dedent(inspect.getsource(m.det_bareiss))
    assert old in src
    ns = {"np": np}
    exec(compile(src.replace(old, new), "<mutant>", "exec"), ns)
    assert not _pins_hold(ns["det_bareiss"])


def test_extended_bonus_recovers_the_last_invariant_factors():
    """Section 3.2: with i right-hand sides, pi~ = s~^i / gcd(det(R N), s~^i)
    (N = s~ X) is the product of the i largest invariant factors for random B
    and R (with high probability: a prime q dividing them is lost with
    probability about 1/q, so the factors here are large primes; these
    seeds), checked against the Smith form the matrices are built with, and
    it divides det(A)."""
    import math

    for n, tail, seed in ((12, [101, 101 * 103, 101 * 103 * 107], 1),
                          (16, [113, 113 * 127, 113 * 127 * 131, 113 * 127 * 131 * 137], 2)):
        s_list = [1] * (n - len(tail)) + tail
        A, _ = synth.smith_matrix(s_list, seed, 0.3)
        d = oracle.det_bareiss(A)
        rng = np.random.default_rng(seed)
        for i in (1, 2, 3):
            B = rng.integers(0, 100, size=(n, i))
            R = rng.integers(1, 1 << 16, size=(i, n))
            s, pi = oracle.extended_bonus(A, B, R)
            assert s == s_list[-1]
            assert pi == math.prod(s_list[-i:])
            assert d % pi == 0


def test_extended_bonus_with_one_right_hand_side_is_s_n():
    """i = 1: pi~ = s~ / gcd(r . N, s~), which is s~ itself for a random
    combination r (Alg. 4.1 sets pi~_1 = s~_n)."""
    A = synth.dense_uniform(10, -20, 20, 44)
    rng = np.random.default_rng(44)
    B = rng.integers(0, 50, size=(10, 1))
    R = rng.integers(1, 1 << 16, size=(1, 10))
    s, pi = oracle.extended_bonus(A, B, R)
    _, den = oracle.solve_rational(A, B[:, 0])
    assert s == den and pi == s
