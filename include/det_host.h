/*
 * det_host.h -- the host-side steps of the introspective determinant,
 * exported so that they can be checked on a machine without a GPU.  None of
 * these functions touches the device.
 *
 * Integers cross this boundary as (sign, little-endian base-2^32 limbs);
 * sign is -1, 0 or +1 and a zero value has no limbs.  Output buffers belong
 * to the caller; when `cap` limbs are not enough the call returns
 * DET_E_BUFFER_TOO_SMALL and writes the needed count to *len.
 */
#ifndef PAPER_CS_0511066_AMD_DET_HOST_H
#define PAPER_CS_0511066_AMD_DET_HOST_H

#include <stdint.h>

#include "det.h"

#ifdef __cplusplus
extern "C" {
#endif

/* 1 if q is prime (deterministic Miller-Rabin, complete for 32-bit q), else 0. */
int det_host_is_prime(uint32_t q);

/* count distinct random primes in (2^(bits-1), 2^bits), 12 <= bits <= 31,
 * drawn uniformly without replacement from the seeded stream (Alg. 2.1 draws
 * each p_i uniformly from the remaining prime set). */
det_status det_host_sample_primes(uint64_t seed, int bits, int64_t count, uint32_t *out);

/* log2 of Hadamard's bound for |det A| (Lemma 2.1), rounded up: the smaller
 * of the row and column forms prod ||a||_2.  A: host, row-major n x n int64. */
double det_host_hadamard_log2(const int64_t *A, int64_t n, int64_t lda);

/* Run length of unchanged reconstructions required by Lemma 2.1(iv) for
 * failure probability 2^-log2_inv_eps, primes drawn from (2^(bits-1), 2^bits)
 * and a bound of logl_H base-l digits.  -1 if the prime set is too small. */
int64_t det_host_et_run_length(double log2_inv_eps, int bits, double logl_H);

/* Chinese remaindering in the symmetric range (Section 2.1): the r with
 * r = residues[i] (mod primes[i]) and -floor(M/2) <= r < ceil(M/2), M the
 * product of the (distinct odd) primes, added in order.  *same_run: number
 * of trailing primes that left r unchanged (the early-termination counter). */
det_status det_host_crt(const uint32_t *residues, const uint32_t *primes, int64_t count, int *sign,
                        uint32_t *mag, int64_t cap, int64_t *len, int64_t *same_run);

/* Rational reconstruction: a/d with a = u d (mod m), |a| <= 2^Nbits,
 * 0 < d <= 2^Dbits, gcd(a, d) = 1 (u, m > 0 given as magnitudes).
 * prime_base: 0 for a general m; a prime q when m is a power of q (then the
 * coprimality test is q not dividing d, as in the p-adic lifting).
 * DET_E_INVALID when no such fraction exists. */
det_status det_host_ratrecon(const uint32_t *u, int64_t ulen, const uint32_t *m, int64_t mlen,
                             int64_t Nbits, int64_t Dbits, uint64_t prime_base, int *a_sign,
                             uint32_t *a_mag, int64_t a_cap, int64_t *a_len, uint32_t *d_mag,
                             int64_t d_cap, int64_t *d_len);

/* Big-integer arithmetic of the reconstruction steps: op 0 a+b, 1 a-b,
 * 2 a*b, 3 floor(a/b), 4 a mod b (b > 0, result in [0, b)), 5 gcd(|a|,|b|). */
det_status det_host_bigint(int op, int a_sign, const uint32_t *a, int64_t alen, int b_sign,
                           const uint32_t *b, int64_t blen, int *out_sign, uint32_t *out,
                           int64_t cap, int64_t *out_len);

/* The extended bonus of Section 3.2 (Alg. 4.1 with m solvings) from the
 * p-adic expansions of the m x m combinations y[h][a] = R_a . x_h, with
 * x_h = A^{-1} b_h, lifted modulo np distinct primes p_z (np = 1: one
 * lifting; np > 1: liftings side by side, Section 6):
 * comb[((h*m + a)*np + z)*k + i] = R_a . (digit i of x_h modulo p_z), so
 * y[h][a] = sum_{i<k} comb[..+i] p_z^i mod p_z^k (host array, m*m*np*k
 * entries, each < 2^64), and y[h][a] modulo P = prod_z p_z^k by Chinese
 * remaindering.  Every y[h][a] is rebuilt by rational reconstruction
 * (|numerator| <= 2^Nbits, 0 < denominator <= 2^Dbits; needs
 * Nbits + Dbits + 1 < log2 P).  Outputs, as magnitudes:
 *   s~  = lcm of the denominators found (a divisor of s_n),
 *   pi~ = s~^m / gcd(det(R N), s~^m) with R N = s~ (R_a . x_h), a divisor of
 *         s_n s_{n-1} ... s_{n-m+1};
 * *failed = number of combinations whose reconstruction failed (then pi~ = 1
 * and s~ covers only the others).  1 <= m <= 64, 1 <= np <= 4. */
det_status det_host_extended_bonus(const uint64_t* comb, int64_t m, int64_t k,
                                   const uint32_t* primes, int64_t np, int64_t Nbits,
                                   int64_t Dbits, uint32_t* s_mag, int64_t s_cap, int64_t* s_len,
                                   uint32_t* pi_mag, int64_t pi_cap, int64_t* pi_len,
                                   int64_t* failed);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_CS_0511066_AMD_DET_HOST_H */
