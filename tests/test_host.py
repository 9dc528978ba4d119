"""CPU tests of the library's host side (no GPU needed): the shared library
loads and exports every function the headers declare, and the host steps of
the method agree with the oracle and with Python integers."""
import math
import os
import random
import re

import numpy as np
import pytest

import oracle
import synth
from conftest import ROOT, test_primes

det = pytest.importorskip("paper_cs_0511066_amd")


def _declared_functions():
    names = []
    for h in ("det.h", "det_host.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"\b(det_[a-z0-9_]+|dixon_lift[a-z_]*)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert "det_mod_primes" in names and "dixon_lift" in names and "det_introspective" in names
    for name in names:
        assert hasattr(det._lib, name), name
    assert set(names) == set(det.EXPORTED)


def test_status_strings():
    assert det._lib.det_status_str(0) == b"DET_OK"
    assert det._lib.det_status_str(4) == b"DET_E_SINGULAR_MOD_P"


def test_is_prime_matches_sympy():
    sympy = pytest.importorskip("sympy")
    rng = random.Random(1)
    cases = list(range(0, 3000)) + [rng.randrange(1 << 20, 1 << 32) for _ in range(3000)]
    cases += [4294967291, 4294967295, 2147483647, 25326001, 3215031751, 4759123141 % (1 << 32)]
    for q in cases:
        assert det.det_host_is_prime(q) == bool(sympy.isprime(q)), q


@pytest.mark.parametrize("bits", [12, 23, 26])
def test_sample_primes(bits):
    ps = det.det_host_sample_primes(42, bits, 200)
    assert len(set(ps.tolist())) == 200
    lo, hi = 1 << (bits - 1), 1 << bits
    assert all(lo < p < hi and oracle.is_prime(int(p)) for p in ps)
    assert np.array_equal(ps, det.det_host_sample_primes(42, bits, 200))
    assert not np.array_equal(ps, det.det_host_sample_primes(43, bits, 200))


def test_bigint_against_python_ints():
    rng = random.Random(7)
    vals = [0, 1, -1, 2 ** 64, -(2 ** 64) + 1, 2 ** 127 - 1, 3 ** 200, -(7 ** 150)]
    vals += [rng.randrange(-(1 << 4000), 1 << 4000) for _ in range(30)]
    vals += [rng.randrange(-(1 << 200), 1 << 200) for _ in range(30)]
    for a in vals:
        for b in rng.sample(vals, 8):
            assert det.det_host_bigint("add", a, b) == a + b
            assert det.det_host_bigint("sub", a, b) == a - b
            assert det.det_host_bigint("mul", a, b) == a * b
            if b > 0:
                assert det.det_host_bigint("floordiv", a, b) == a // b
                assert det.det_host_bigint("mod", a, b) == a % b
            assert det.det_host_bigint("gcd", a, b) == math.gcd(a, b)


def test_bigint_karatsuba_sizes():
    rng = random.Random(8)
    for bits in (3000, 3100, 6400, 20000, 65000):
        a = rng.getrandbits(bits) | 1
        b = -rng.getrandbits(bits - 17)
        assert det.det_host_bigint("mul", a, b) == a * b


def test_bigint_division_edge_cases():
    # quotient digit estimates that need the add-back step of long division
    for a, b in [((1 << 192) - 1, (1 << 128) - 1), (1 << 256, (1 << 128) + 1),
                 ((1 << 255) + (1 << 191), (1 << 127) + 1), (2 ** 400 - 2 ** 300, 2 ** 200 - 1)]:
        assert det.det_host_bigint("floordiv", a, b) == a // b
        assert det.det_host_bigint("mod", a, b) == a % b
        assert det.det_host_bigint("floordiv", -a, b) == -a // b


def test_crt_matches_oracle():
    rng = random.Random(3)
    for count in (1, 2, 5, 40):
        ps = test_primes(1 << 22, 1 << 26, count, count)
        rs = [rng.randrange(p) for p in ps]
        r, _ = det.det_host_crt(rs, ps)
        assert r == oracle.crt_symmetric(rs, ps)[0]


def test_crt_same_run_counts_unchanged_primes():
    ps = test_primes(1 << 22, 1 << 23, 10, 5)
    target = -987654321987
    rs = [target % p for p in ps]
    r, same = det.det_host_crt(rs, ps)
    assert r == target
    # target needs 2 primes (|target| < 2^40 < p0 p1 / 2), the other 8 leave it unchanged
    assert same == 8
    out = oracle.et_cra(rs, ps, 4000, k=8)
    assert out == (target, 10, True)


def test_ratrecon_matches_oracle():
    rng = random.Random(11)
    p = 33554393
    for k in (3, 10, 40):
        m = p ** k
        half = (m.bit_length() - 2) // 2
        for _ in range(20):
            d = rng.randrange(1, 1 << half)
            a = rng.randrange(-(1 << half), 1 << half)
            g = math.gcd(a, d)
            a, d = a // g, d // g
            u = a * pow(d, -1, m) % m
            got = det.det_host_ratrecon(u, m, half, half)
            assert got == (a, d)
            assert got == oracle.rational_reconstruct(u, m, 1 << half, 1 << half)


def test_ratrecon_lehmer_large_prime_power():
    """p-adic sizes of the lifting (tens of thousands of bits): the Lehmer
    batches must stop exactly at the first remainder <= N."""
    rng = random.Random(12)
    p = 33554393
    for k in (200, 900):
        m = p ** k
        half = (m.bit_length() - 2) // 2
        for trial in range(4):
            d = rng.randrange(1, 1 << half)
            if d % p == 0:
                d += 1
            a = rng.randrange(-(1 << half), 1 << half)
            g = math.gcd(a, d)
            a, d = a // g, d // g
            u = a * pow(d, -1, m) % m
            assert det.det_host_ratrecon(u, m, half, half, prime_base=p) == (a, d)
            assert det.det_host_ratrecon(u, m, half, half) == (a, d)
    # bounds just tight enough: numerator and denominator of equal size
    m = p ** 50
    d, a = (1 << 600) + 12345, -((1 << 599) + 777)
    u = a * pow(d, -1, m) % m
    assert det.det_host_ratrecon(u, m, 601, 601, prime_base=p) == \
        oracle.rational_reconstruct(u, m, 1 << 601, 1 << 601)


def test_ratrecon_random_against_oracle():
    """The Lehmer passes, the leading-bit quotient steps and the full
    divisions of the host reconstruction against the textbook extended
    Euclid: random moduli (general and prime powers) from 64 to 5000 bits,
    residues of every magnitude (tiny ones give huge first quotients), and
    bounds on both sides of 2 N D < m; the outputs must be identical,
    failures included."""
    rng = random.Random(19)
    cases = 0
    for trial in range(300):
        bits = rng.choice([64, 200, 700, 2000, 5000])
        if trial % 3 == 0:
            p = rng.choice([33554393, 16777213, 10007])
            m = p ** max(1, bits // p.bit_length())
        else:
            m = rng.getrandbits(bits) | (1 << (bits - 1)) | 1
        u = rng.randrange(1, m) >> rng.choice([0, 0, 0, 5, 60, bits // 2])
        half = (m.bit_length() - 2) // 2
        Nbits = max(1, half + rng.randint(-40, 40))
        Dbits = max(1, half + rng.randint(-40, 40))
        got = det.det_host_ratrecon(u, m, Nbits, Dbits)
        ref = oracle.rational_reconstruct(u, m, 1 << Nbits, 1 << Dbits)
        assert got == ref, (trial, bits, Nbits, Dbits)
        cases += ref is not None
    assert cases > 20


def test_ratrecon_rejects_when_out_of_bounds():
    m = 10007 ** 2
    u = 123456 * pow(654321, -1, m) % m
    got = det.det_host_ratrecon(u, m, 5, 5)
    ref = oracle.rational_reconstruct(u, m, 32, 32)
    assert got == ref


def test_hadamard_log2_upper_bound():
    for n, lo, hi, seed in ((10, -100, 100, 1), (64, -100, 100, 2), (50, 0, 255, 3)):
        A = synth.dense_uniform(n, lo, hi, seed)
        h = det.det_host_hadamard_log2(A)
        exact = 0.5 * math.log2(oracle.hadamard_sq(A))
        assert exact <= h <= exact + 1e-5
        assert abs(oracle.det_bareiss(A)).bit_length() - 1 <= h


def test_et_run_length_matches_lemma():
    for eps, bits, L in ((64, 23, 568.0), (64, 23, 3.0), (20, 16, 30.0)):
        P = (1 << (bits - 1)) / math.log(1 << bits)
        assert det.det_host_et_run_length(eps, bits, L) == oracle.et_k(eps, P, math.ceil(L)) or \
            det.det_host_et_run_length(eps, bits, L) >= oracle.et_k(eps, P, math.ceil(L))
        k = det.det_host_et_run_length(eps, bits, L)
        assert (L / (P - math.ceil(L))) ** k <= 2.0 ** -eps * (1 + 1e-9)


def test_context_without_gpu_reports_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(det.DetError) as e:
        det.Context(0)
    assert e.value.status == 8


def _bonus_inputs(n, tail, seed, m, p):
    """A Smith-form matrix with the given last invariant factors, m seeded
    right-hand sides and combination vectors, and the m x m x k combination
    digits R_a . x_{h,i} formed from the oracle's Dixon digits."""
    s = [1] * (n - len(tail)) + list(tail)
    A, _ = synth.smith_matrix(s, seed, None)
    rng = np.random.default_rng(seed)
    B = rng.integers(0, 64, size=(n, m), dtype=np.int64)
    R = rng.integers(1, 1 << 16, size=(m, n), dtype=np.int64)
    hb = oracle.hadamard_bits(A)
    bmax = max(math.isqrt(int(sum(int(v) ** 2 for v in B[:, h]))) + 1 for h in range(m))
    Nbits = int(R.sum(axis=1).max()).bit_length() + hb + bmax.bit_length() + 1
    Dbits = hb
    k = -(-(Nbits + Dbits + 2) // (p.bit_length() - 1)) + 1
    comb = np.zeros((m, m, k), dtype=np.uint64)
    for h in range(m):
        X = oracle.dixon_digits(A, B[:, h], p, k)          # k x n, in [0, p)
        for a in range(m):
            comb[h, a] = (X @ R[a]).astype(np.uint64)      # < 2^16 * 2^25 * n: exact
    return A, B, R, comb, Nbits, Dbits, s


@pytest.mark.parametrize("n,tail,seed,m", [(60, [101, 101 * 103], 31, 2),
                                           (96, [107, 107 * 109, 107 * 109 * 113], 32, 3),
                                           (40, [1, 1], 33, 2)])
def test_extended_bonus_host_matches_oracle(n, tail, seed, m):
    """The host step of the extended bonus (Section 3.2) on combination
    digits built from the oracle's Dixon digits: s~ and pi~ equal those the
    oracle computes from the exact rational solutions, and lcm(s~, pi~)
    divides det(A)."""
    p = test_primes(1 << 24, 1 << 25, 1, seed)[0]
    A, B, R, comb, Nbits, Dbits, s = _bonus_inputs(n, tail, seed, m, p)
    got_s, got_pi, failed = det.det_host_extended_bonus(comb, p, Nbits, Dbits)
    ref_s, ref_pi = oracle.extended_bonus(A, B, R)
    assert failed == 0
    assert (got_s, got_pi) == (ref_s, ref_pi)
    d = math.prod(s)
    assert d % math.lcm(got_s, got_pi) == 0
    if tail[-1] > 1:                    # the m largest invariant factors, found exactly
        assert got_pi == math.prod(s[-m:])


@pytest.mark.parametrize("n,tail,seed,m,count", [(60, [101, 101 * 103], 31, 2, 2),
                                                 (96, [107, 107 * 109, 107 * 109 * 113], 32, 3, 3),
                                                 (40, [1, 1], 33, 2, 4)])
def test_extended_bonus_host_several_primes(n, tail, seed, m, count):
    """Liftings modulo several primes side by side (Section 6), each only
    long enough for its share of the bound: the combinations are rebuilt by
    Chinese remaindering of the p-adic values, and s~, pi~ equal the oracle's;
    any single prime's digits are too short on their own."""
    ps = test_primes(1 << 24, 1 << 25, count, seed + 7)
    A, B, R, _, Nbits, Dbits, s = _bonus_inputs(n, tail, seed, m, ps[0])
    log2P = sum(math.log2(p) for p in ps)
    k = int(math.ceil((Nbits + Dbits + 2) / log2P)) + 1
    comb = np.zeros((m, m, count, k), dtype=np.uint64)
    for h in range(m):
        for z, p in enumerate(ps):
            X = oracle.dixon_digits(A, B[:, h], p, k)
            for a in range(m):
                comb[h, a, z] = (X @ R[a]).astype(np.uint64)
    got_s, got_pi, failed = det.det_host_extended_bonus(comb, ps, Nbits, Dbits)
    ref_s, ref_pi = oracle.extended_bonus(A, B, R)
    assert failed == 0
    assert (got_s, got_pi) == (ref_s, ref_pi)
    assert math.prod(s) % math.lcm(got_s, got_pi) == 0


def test_padic_remaindering_rebuilds_a_fraction():
    """Chinese remaindering of p-adic expansions: the expansions of a known
    fraction a/d modulo p1^k and p2^k, fed as digit sums (m = 1, R = 1),
    give back d as s~ = pi~; the digits are those of Python's exact modular
    arithmetic, so nothing of the library enters the expected value."""
    ps = test_primes(1 << 24, 1 << 25, 2, 91)
    k = 40                                           # 2 x 40 x 24 bits > 2 x 900 + 2
    a, d = -(3 ** 500) + 17, 7 ** 300 + 2
    assert math.gcd(a, d) == 1 and all(d % p for p in ps)
    comb = np.zeros((1, 1, 2, k), dtype=np.uint64)
    for z, p in enumerate(ps):
        v = a * pow(d, -1, p ** k) % p ** k
        for i in range(k):
            comb[0, 0, z, i] = v % p
            v //= p
    got_s, got_pi, failed = det.det_host_extended_bonus(comb, ps, 900, 900)
    assert failed == 0 and got_s == d and got_pi == d
    # either prime's 40 digits alone (960 bits) cannot determine a/d (|a| d
    # needs 1636): the reconstruction fails or finds another fraction
    for z in range(2):
        one_s, _, one_failed = det.det_host_extended_bonus(comb[:, :, z:z + 1], ps[z:z + 1], 900, 900)
        assert one_failed == 1 or one_s != d
    # the remaindering in the other order gives the same value
    got_s2, _, _ = det.det_host_extended_bonus(comb[:, :, ::-1], ps[::-1], 900, 900)
    assert got_s2 == d


def test_extended_bonus_host_reports_a_corrupted_lifting():
    """A wrong digit in one combination's expansion makes its reconstruction
    fail (the bounds leave no room for a spurious fraction), and the failure
    is reported instead of entering pi~."""
    p = test_primes(1 << 24, 1 << 25, 1, 5)[0]
    A, B, R, comb, Nbits, Dbits, s = _bonus_inputs(60, [101, 101 * 103], 31, 2, p)
    bad = comb.copy()
    bad[1, 0, bad.shape[2] // 2] ^= np.uint64(1 << 7)
    _, got_pi, failed = det.det_host_extended_bonus(bad, p, Nbits, Dbits)
    assert failed >= 1 and got_pi == 1
