// Host-side numerics of the method: prime sampling, the Hadamard bound,
// early-terminated Chinese remaindering, rational reconstruction.
#pragma once
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <unordered_set>
#include <vector>

#include "bigint.hpp"

namespace dethost {

// ---------------------------------------------------------------- primes
inline uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
inline uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, a, m);
    a = mulmod64(a, a, m);
    e >>= 1;
  }
  return r;
}
// Deterministic Miller-Rabin for 32-bit n (bases 2, 7, 61 are a complete
// witness set below 4,759,123,141).
inline bool is_prime_u32(uint32_t n) {
  if (n < 2) return false;
  for (uint32_t q : {2u, 3u, 5u, 7u, 11u, 13u, 61u})
    if (n % q == 0) return n == q;
  uint32_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; s++; }
  for (uint64_t a : {2ull, 7ull, 61ull}) {
    uint64_t x = powmod64(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; r++) {
      x = mulmod64(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

inline uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Uniform random primes in (2^(bits-1), 2^bits), without replacement
// (Alg. 2.1 draws each p_i uniformly from the remaining set P).  Rejection
// sampling: draw a uniform integer of the interval, keep it if prime and unused.
struct PrimeSampler {
  uint64_t state;
  int bits;
  std::unordered_set<uint32_t> used;
  PrimeSampler(uint64_t seed, int b) : state(seed), bits(b) {}
  uint32_t next() {
    const uint64_t lo = 1ull << (bits - 1), span = 1ull << (bits - 1);
    for (;;) {
      uint32_t c = (uint32_t)(lo + splitmix64(state) % span) | 1u;
      if (c <= lo || c >= 2 * lo) continue;
      if (!is_prime_u32(c) || used.count(c)) continue;
      used.insert(c);
      return c;
    }
  }
};

// Number of primes in (l, 2l), l = 2^(bits-1), rounded down: l / ln(2l)
// (an under-estimate of pi(2l) - pi(l) for these l, so the early
// termination run length computed from it is on the safe side).
inline double prime_set_size(int bits) {
  const double l = ldexp(1.0, bits - 1);
  return l / log(2.0 * l);
}

// ---------------------------------------------------------------- bounds
// log2 of Hadamard's bound, min over the row and column forms
// (|det A| <= prod_j ||a_j||_2), from per-column and per-row sums of
// squares.  Each sum is rounded upward by a relative margin that covers the
// double rounding of n additions, so the result is an upper bound.
struct Bounds {
  double log2_h = 0;        // log2 H (min of the two forms)
  double log2_hcol = 0;     // log2 of the column form
  double log2_min_col = 0;  // log2 min_j ||a_j||_2
  double amax = 0;          // ||A|| = max |a_ij|
};
inline Bounds bounds_from_sums(const std::vector<double>& colsq, const std::vector<double>& rowsq,
                               double amax) {
  Bounds b;
  const double up = 1.0 + 1e-12;
  double lc = 0, lr = 0, mincol = INFINITY;
  for (double v : colsq) {
    if (v <= 0) { lc = -INFINITY; mincol = 0; break; }
    lc += 0.5 * log2(v * up);
    mincol = fmin(mincol, v);
  }
  for (double v : rowsq) {
    if (v <= 0) { lr = -INFINITY; break; }
    lr += 0.5 * log2(v * up);
  }
  const size_t n = colsq.size();
  const double slack = 1e-9 * (double)n + 1e-6;   // covers the log2 rounding
  b.log2_hcol = lc + slack;
  b.log2_h = fmin(lc, lr) + slack;
  b.log2_min_col = mincol > 0 ? 0.5 * log2(mincol) - slack : 0;
  b.amax = amax;
  if (!(b.log2_h > 0)) b.log2_h = 0;    // H < 1 only when det = 0 or n = 0
  if (!(b.log2_hcol > 0)) b.log2_hcol = 0;
  return b;
}
inline Bounds bounds_host(const int64_t* A, int64_t n, int64_t lda) {
  std::vector<double> colsq(n, 0.0), rowsq(n, 0.0);
  double amax = 0;
  for (int64_t i = 0; i < n; i++)
    for (int64_t j = 0; j < n; j++) {
      const double a = (double)A[i * lda + j];
      colsq[j] += a * a;
      rowsq[i] += a * a;
      amax = fmax(amax, fabs(a));
    }
  return bounds_from_sums(colsq, rowsq, amax);
}

// ---------------------------------------------------------------- CRT
// Incremental Chinese remaindering in the symmetric range (Section 2.1:
// r_t is reconstructed modulo p_0...p_t with -floor(M/2) <= r_t < ceil(M/2)).
// Garner step with a centred correction digit t: if r is in the symmetric
// range mod M (M odd), r + M t is in the symmetric range mod M p.
struct CrtState {
  BigInt r, M;
  int64_t count = 0;
  int64_t same = 0;     // consecutive primes that left r unchanged
  // Adds residue d (in [0, p)) of an odd prime p; returns true if r_t = r_{t-1}.
  bool add(uint32_t p, uint32_t d) {
    if (count == 0) {
      int64_t c = d > (p - 1) / 2 ? (int64_t)d - p : (int64_t)d;
      r = BigInt::from_i64(c);
      M = BigInt::from_u64(p);
      count = 1;
      same = 0;
      return false;
    }
    const uint64_t rm = r.mod_small(p);
    bool unchanged = rm == d;
    if (!unchanged) {
      const uint64_t mm = M.mod_small(p);
      const uint64_t inv = powmod64(mm, p - 2, p);
      uint64_t t = mulmod64((d + p - rm) % p, inv, p);
      int64_t tc = t > (p - 1) / 2 ? (int64_t)t - p : (int64_t)t;
      r = r + M * BigInt::from_i64(tc);
    }
    M.mul_add_small(p, 0);
    count++;
    same = unchanged ? same + 1 : 0;
    return unchanged;
  }
};

// Lemma 2.1(iv): the run of unchanged reconstructions that bounds the
// failure probability by eps: k = ceil(log(1/eps) / (log P' - log log_l H)),
// P' = |P| - ceil(log_l H).  Returns -1 if |P| is too small for the lemma.
inline int64_t et_run_length(double log2_inv_eps, double P_size, double logl_H) {
  const double Pp = P_size - ceil(logl_H);
  const double den = log2(Pp) - log2(fmax(logl_H, 1.0));
  if (!(Pp > 0) || !(den > 0)) return -1;
  return (int64_t)fmax(1.0, ceil(log2_inv_eps / den));
}

// ---------------------------------------------------------------- rational reconstruction
// Bits [s, s + 63) of a non-negative BigInt.
inline uint64_t top_bits(const BigInt& v, int64_t s) {
  const size_t w = (size_t)(s / 64);
  const int sh = (int)(s % 64);
  uint64_t lo = w < v.mag.size() ? v.mag[w] : 0;
  uint64_t hi = w + 1 < v.mag.size() ? v.mag[w + 1] : 0;
  uint64_t x = sh ? (lo >> sh) | (hi << (64 - sh)) : lo;
  return x & ((1ull << 63) - 1);
}

// Bits [s, s + 126) of |v|.
inline u128 top_bits126(const BigInt& v, int64_t s) {
  const u128 lo = top_bits(v, s), hi = top_bits(v, s + 63);
  return lo | (hi << 63);
}

// Quotient floor(a / b) for 0 <= a < 2^126, 0 < b (128-bit): by comparison
// when it is below 4 (most quotients of the Euclidean algorithm are 1, 2 or
// 3), else from the operands in double precision (relative error below
// 2^-50, so an estimate below 2^50 is within one of the quotient), corrected
// exactly; a 128-bit division only for larger quotients.
inline __int128 small_quot(__int128 a, __int128 b) {
  if (a < b) return 0;
  if (a < 2 * b) return 1;
  if (a < 3 * b) return 2;
  if (a < 4 * b) return 3;
  constexpr double TWO64 = 18446744073709551616.0;
  const double da = (double)(uint64_t)((u128)a >> 64) * TWO64 + (double)(uint64_t)a;
  const double db = (double)(uint64_t)((u128)b >> 64) * TWO64 + (double)(uint64_t)b;
  const double qd = da / db;
  if (qd < 1e15) {
    int64_t q = (int64_t)qd;
    __int128 r = a - (__int128)q * b;
    while (r < 0) {
      q--;
      r += b;
    }
    while (r >= b) {
      q++;
      r -= b;
    }
    return q;
  }
  return a / b;
}

// det(M) of a small square BigInt matrix by fraction-free (Bareiss)
// elimination: every division is exact; a zero pivot is replaced by a row
// below it (changing the sign).
inline BigInt bareiss_det(std::vector<std::vector<BigInt>> M) {
  const size_t n = M.size();
  if (n == 0) return BigInt::from_i64(1);
  int sign = 1;
  BigInt prev = BigInt::from_i64(1);
  for (size_t k = 0; k < n; k++) {
    if (M[k][k].is_zero()) {
      size_t r = k + 1;
      while (r < n && M[r][k].is_zero()) r++;
      if (r == n) return BigInt();
      std::swap(M[k], M[r]);
      sign = -sign;
    }
    for (size_t i = k + 1; i < n; i++)
      for (size_t j = k + 1; j < n; j++)
        M[i][j] = BigInt::div_exact(M[i][j] * M[k][k] - M[i][k] * M[k][j], prev);
    prev = M[k][k];
  }
  BigInt d = M[n - 1][n - 1];
  if (sign < 0) d = -d;
  return d;
}

// The integer sum_i c[i] p^i (c[i] < 2^64, p < 2^25) and p^k, for the
// rational reconstruction of a p-adic expansion: Horner's rule two digits a
// pass (multiplier p^2, a 128-bit addend), p^k by squaring.
inline void radix_value(const uint64_t* c, int64_t k, uint64_t p, BigInt& y, BigInt& pk) {
  y = BigInt();
  int64_t i = k - 1;
  if (k & 1) {
    y = BigInt::from_u64(c[k - 1]);
    i = k - 2;
  }
  const uint64_t p2 = p * p;
  for (; i >= 1; i -= 2) y.mul_add_u128(p2, (u128)c[i] * p + c[i - 1]);
  pk = BigInt::from_i64(1);
  BigInt b = BigInt::from_u64(p);
  for (int64_t e = k; e > 0; e >>= 1) {
    if (e & 1) pk = pk * b;
    if (e > 1) b = b * b;
  }
}

// Find a/d with a = u d (mod m), |a| <= N, 0 < d <= D, gcd(a, d) = 1, unique
// when 2 N D < m: the extended Euclidean algorithm on (m, u mod m), stopped
// at the first remainder <= N.  The remainder sequence is advanced with
// Lehmer's method (Knuth, TAOCP 4.5.2, Algorithm L, on two words: the
// quotients of the leading 126 bits, accepted while both bracketing quotients
// agree and the cofactors stay below 2^62, give a 2x2 cofactor matrix applied
// to the full numbers in one pass) while the remainder is more than 130 bits
// above N, so no batch can step past the stopping point; the last steps are
// plain divisions.  When m is a power of the prime
// `pbase` (pbase != 0), any common factor of the result lies in m, so
// gcd(a, d) = 1 reduces to pbase not dividing d.
inline bool rational_reconstruct(const BigInt& u_in, const BigInt& m, const BigInt& N,
                                 const BigInt& D, BigInt& a_out, BigInt& d_out,
                                 const uint64_t* pbases, int nbases) {
  BigInt q, u;
  BigInt::divmod_floor(u_in, m, q, u);
  BigInt r0 = m, r1 = u, t0, t1 = BigInt::from_i64(1);
  const int64_t nbits = N.bit_length();
  while (r1.cmp(N) > 0) {
    if (r1.bit_length() > nbits + 130) {
      // Lehmer (double-word): the quotients of the leading 126 bits, as long
      // as both bracketing quotients agree and the cofactors stay below
      // 2^62, taken as one 2 x 2 cofactor matrix
      const int64_t s = std::max<int64_t>(0, r0.bit_length() - 126);
      __int128 x = (__int128)top_bits126(r0, s), y = (__int128)top_bits126(r1, s);
      __int128 A = 1, B = 0, C = 0, Dd = 1;
      const __int128 lim = (__int128)1 << 62;
      while (y + C > 0 && y + Dd > 0 && x + A >= 0 && x + B >= 0) {
        const __int128 qa = small_quot(x + A, y + C), qb = small_quot(x + B, y + Dd);
        if (qa != qb) break;
        const __int128 nC = A - qa * C, nD = B - qa * Dd;
        if (nC >= lim || nC <= -lim || nD >= lim || nD <= -lim) break;
        A = C; C = nC;
        B = Dd; Dd = nD;
        const __int128 T = x - qa * y; x = y; y = T;
      }
      if (B != 0) {
        BigInt::lincomb2(r0, r1, (int64_t)A, (int64_t)B, (int64_t)C, (int64_t)Dd);
        BigInt::lincomb2(t0, t1, (int64_t)A, (int64_t)B, (int64_t)C, (int64_t)Dd);
        continue;
      }
    }
    // one Euclidean step.  When r1 is within 31 bits of r0, the quotient q
    // (below 2^31) is within one of qe = floor(xh / yh) from the leading 63
    // bits: (r0, r1) <- (r1, r0 - (qe - 1) r1) in place, then r1 -= r0 while
    // r1 >= r0 (at most twice), and the same step on the cofactors.
    const int64_t sh = std::max<int64_t>(0, r0.bit_length() - 63);
    const uint64_t xh = top_bits(r0, sh), yh = top_bits(r1, sh);
    if (yh >= (1ull << 32)) {
      int64_t q = (int64_t)(xh / yh);
      if (q > 0) q--;
      BigInt::lincomb2(r0, r1, 0, 1, 1, -q);
      while (r1.cmp(r0) >= 0) {
        BigInt::lincomb2(r0, r1, 1, 0, -1, 1);
        q++;
      }
      BigInt::lincomb2(t0, t1, 0, 1, 1, -q);
      continue;
    }
    BigInt qq, rr;
    BigInt::divmod_floor(r0, r1, qq, rr);
    r0 = r1;
    r1 = rr;
    BigInt t2 = t0 - qq * t1;
    t0 = t1;
    t1 = t2;
  }
  BigInt a = r1, d = t1;
  if (d.is_zero()) return false;
  if (d.sign < 0) { a = -a; d = -d; }
  if (d.cmp(D) > 0) return false;
  if (nbases > 0) {
    for (int z = 0; z < nbases; z++)
      if (d.mod_small(pbases[z]) == 0) return false;
  } else if (!(BigInt::gcd(a, d).cmp(BigInt::from_i64(1)) == 0)) {
    return false;
  }
  a_out = a;
  d_out = d;
  return true;
}

inline bool rational_reconstruct(const BigInt& u_in, const BigInt& m, const BigInt& N,
                                 const BigInt& D, BigInt& a_out, BigInt& d_out,
                                 uint64_t pbase = 0) {
  return rational_reconstruct(u_in, m, N, D, a_out, d_out, &pbase, pbase ? 1 : 0);
}

// u^{-1} mod m for m a power of the prime q (false when q divides u): the
// extended Euclidean algorithm run down to the remainder 1, which is the
// rational reconstruction with numerator bound 1 (the cofactor d of the
// remainder +-1 satisfies +-1 = d u mod m).
inline bool inverse_mod_prime_power(const BigInt& u, const BigInt& m, uint64_t q, BigInt& inv) {
  BigInt a, d;
  if (!rational_reconstruct(u, m, BigInt::from_i64(1), m, a, d, q)) return false;
  if (a.sign < 0) d = m - d;
  inv = d;
  return true;
}

// Chinese remaindering of p-adic values (several liftings in parallel,
// Section 6): P_z = p_z^k for distinct primes p_z, and y = the integer in
// [0, P_0 ... P_{np-1}) with y = y_z mod P_z, by Garner's mixed-radix form
// y = v_0 + P_0 (v_1 + P_1 (...)) with
//   v_z = (y_z - (v_0 + P_0 v_1 + ... )) (P_0 ... P_{z-1})^{-1} mod P_z.
// The inverses depend only on the primes and k, so setup() can run before
// the digits exist.
struct PadicCrt {
  int np = 0;
  std::vector<uint64_t> p;
  std::vector<BigInt> P, inv;                   // inv[z] = (P_0 ... P_{z-1})^{-1} mod P_z
  BigInt M;                                     // P_0 ... P_{np-1}
  bool setup(const uint32_t* ps, int count, int64_t k) {
    np = count;
    p.assign(ps, ps + count);
    P.assign(count, BigInt());
    inv.assign(count, BigInt());
    M = BigInt::from_i64(1);
    for (int z = 0; z < count; z++) {
      BigInt pk = BigInt::from_i64(1), b = BigInt::from_u64(ps[z]);
      for (int64_t e = k; e > 0; e >>= 1) {
        if (e & 1) pk = pk * b;
        if (e > 1) b = b * b;
      }
      P[z] = pk;
      if (z > 0) {
        BigInt q, r;
        BigInt::divmod_floor(M, pk, q, r);
        if (!inverse_mod_prime_power(r, pk, ps[z], inv[z])) return false;   // (equal primes)
      }
      M = M * pk;
    }
    return true;
  }
  // y from the values y_z (any integers; each is reduced mod P_z first)
  BigInt combine(const BigInt* y) const {
    BigInt q, acc, Mz = BigInt::from_i64(1);
    for (int z = 0; z < np; z++) {
      BigInt v;
      BigInt::divmod_floor(y[z], P[z], q, v);
      if (z > 0) {
        BigInt t;
        BigInt::divmod_floor(v - acc, P[z], q, t);      // (y_z - acc) mod P_z
        BigInt::divmod_floor(t * inv[z], P[z], q, v);
        v = acc + Mz * v;
      }
      acc = v;
      Mz = Mz * P[z];
    }
    return acc;
  }
};

// ---------------------------------------------------------------- extended bonus
// The extended bonus of Section 3.2 (Alg. 4.1 with m >= 2 solvings), from
// the p-adic expansions of the m x m combinations y[h][a] = R_a . x_h,
// x_h = A^{-1} b_h, lifted modulo np primes side by side (np = 1: one
// lifting): comb[((h m + a) np + z) k + i] = R_a . (digit i of x_h modulo
// p_z), so that y[h][a] = sum_i comb[..i] p_z^i (mod p_z^k) for each z, and
// y[h][a] modulo P = prod_z p_z^k by Chinese remaindering.  Each y[h][a] is
// rebuilt by rational reconstruction modulo P (numerator <= 2^Nbits,
// denominator <= 2^Dbits, unique when Nbits + Dbits + 1 < log2 P).
//   s~  = lcm of the denominators of all y[h][a]; every one divides the
//         common denominator of X = [x_0 .. x_{m-1}] and so s_n;
//   R N = s~ R X, the integer m x m matrix with entries num * (s~ / den);
//   pi~ = s~^m / gcd(det(R N), s~^m).
// Since det(R X) P_m is an integer for P_m = s_n s_{n-1} ... s_{n-m+1}
// (Cauchy-Binet over the Smith form of A), s~^m divides det(R N) P_m, so pi~
// divides P_m for any s~ that makes R N integral; and s~ | s_n | P_m, so
// lcm(s~, pi~) divides det(A).  Returns the number of combinations whose
// reconstruction failed (0 on success; then pi~ is set, else pi~ = 1 and s~
// is the lcm of the denominators that were found).  crt: the remaindering
// set up for ps and k (built here when null).
inline int64_t extended_bonus_host(const uint64_t* comb, int m, int64_t k, const uint32_t* ps,
                                   int np, int64_t Nbits, int64_t Dbits, const PadicCrt* crt,
                                   BigInt& s, BigInt& pi) {
  s = BigInt::from_i64(1);
  pi = BigInt::from_i64(1);
  if (m <= 0) return 0;
  PadicCrt own;
  if (!crt) {
    if (!own.setup(ps, np, k)) return (int64_t)m * m;
    crt = &own;
  }
  const BigInt Nb = BigInt::from_i64(1).shl(Nbits), Db = BigInt::from_i64(1).shl(Dbits);
  std::vector<std::vector<BigInt>> num(m, std::vector<BigInt>(m)), den(m, std::vector<BigInt>(m));
  int64_t failed = 0;
  std::vector<BigInt> yz(np);
  BigInt pk;
  for (int h = 0; h < m; h++)
    for (int a = 0; a < m; a++) {
      for (int z = 0; z < np; z++)
        radix_value(comb + (((size_t)h * m + a) * np + z) * k, k, ps[z], yz[z], pk);
      const BigInt y = np == 1 ? yz[0] : crt->combine(yz.data());
      BigInt nu, d;
      if (!rational_reconstruct(y, crt->M, Nb, Db, nu, d, crt->p.data(), np)) {
        failed++;
        continue;
      }
      num[h][a] = nu;
      den[h][a] = d;
      s = BigInt::div_exact(s * d, BigInt::gcd(s, d));
    }
  if (failed) return failed;
  if (m == 1) {
    // one solving: pi~_1 = s~ (Alg. 4.1), no determinant to take
    pi = s;
    return 0;
  }
  // R N (rows a, columns h): exact, as every den divides s~
  std::vector<std::vector<BigInt>> RN(m, std::vector<BigInt>(m));
  for (int a = 0; a < m; a++)
    for (int h = 0; h < m; h++) RN[a][h] = num[h][a] * BigInt::div_exact(s, den[h][a]);
  BigInt sm = BigInt::from_i64(1);
  for (int i = 0; i < m; i++) sm = sm * s;
  BigInt dRN = bareiss_det(RN);
  if (dRN.sign < 0) dRN = -dRN;
  pi = BigInt::div_exact(sm, BigInt::gcd(dRN, sm));
  return 0;
}

inline int64_t extended_bonus_host(const uint64_t* comb, int m, int64_t k, uint64_t p,
                                   int64_t Nbits, int64_t Dbits, BigInt& s, BigInt& pi) {
  const uint32_t p32 = (uint32_t)p;
  return extended_bonus_host(comb, m, k, &p32, 1, Nbits, Dbits, nullptr, s, pi);
}

}  // namespace dethost
