// Host-only entry points (include/det_host.h): thin wrappers around
// bigint.hpp and host_numerics.hpp, the same code the determinant uses.
#include <string.h>

#include <exception>
#include <vector>

#include "../../include/det_host.h"
#include "bigint.hpp"
#include "host_numerics.hpp"

using dethost::BigInt;

namespace {

det_status put(const BigInt& v, int* sign, uint32_t* mag, int64_t cap, int64_t* len) {
  std::vector<uint32_t> l = v.limbs32();
  if (sign) *sign = v.sign;
  *len = (int64_t)l.size();
  if ((int64_t)l.size() > cap) return DET_E_BUFFER_TOO_SMALL;
  if (!l.empty()) memcpy(mag, l.data(), l.size() * sizeof(uint32_t));
  return DET_OK;
}

}  // namespace

extern "C" {

int det_host_is_prime(uint32_t q) { return dethost::is_prime_u32(q) ? 1 : 0; }

det_status det_host_sample_primes(uint64_t seed, int bits, int64_t count, uint32_t* out) {
  if (bits < 12 || bits > 31 || count < 0 || (count > 0 && !out)) return DET_E_INVALID;
  try {
    dethost::PrimeSampler s(seed, bits);
    for (int64_t i = 0; i < count; i++) out[i] = s.next();
    return DET_OK;
  } catch (...) {
    return DET_E_NOMEM;
  }
}

double det_host_hadamard_log2(const int64_t* A, int64_t n, int64_t lda) {
  if (n <= 0 || !A || lda < n) return 0.0;
  return dethost::bounds_host(A, n, lda).log2_h;
}

int64_t det_host_et_run_length(double log2_inv_eps, int bits, double logl_H) {
  return dethost::et_run_length(log2_inv_eps, dethost::prime_set_size(bits), logl_H);
}

det_status det_host_crt(const uint32_t* residues, const uint32_t* primes, int64_t count, int* sign,
                        uint32_t* mag, int64_t cap, int64_t* len, int64_t* same_run) {
  if (count < 0 || !len || !sign || (count > 0 && (!residues || !primes))) return DET_E_INVALID;
  try {
    dethost::CrtState s;
    for (int64_t i = 0; i < count; i++) {
      if (primes[i] < 3 || !(primes[i] & 1) || residues[i] >= primes[i]) return DET_E_INVALID;
      s.add(primes[i], residues[i]);
    }
    if (same_run) *same_run = s.same;
    return put(s.r, sign, mag, cap, len);
  } catch (...) {
    return DET_E_NOMEM;
  }
}

det_status det_host_ratrecon(const uint32_t* u, int64_t ulen, const uint32_t* m, int64_t mlen,
                             int64_t Nbits, int64_t Dbits, uint64_t prime_base, int* a_sign,
                             uint32_t* a_mag, int64_t a_cap, int64_t* a_len, uint32_t* d_mag,
                             int64_t d_cap, int64_t* d_len) {
  if (ulen < 0 || mlen <= 0 || Nbits < 0 || Dbits < 0 || !a_len || !d_len) return DET_E_INVALID;
  try {
    BigInt U = BigInt::from_limbs32(u, (size_t)ulen, 1), M = BigInt::from_limbs32(m, (size_t)mlen, 1);
    if (M.is_zero()) return DET_E_INVALID;
    BigInt a, d;
    if (!dethost::rational_reconstruct(U, M, BigInt::from_i64(1).shl(Nbits),
                                       BigInt::from_i64(1).shl(Dbits), a, d, prime_base))
      return DET_E_INVALID;
    det_status s = put(a, a_sign, a_mag, a_cap, a_len);
    det_status t = put(d, nullptr, d_mag, d_cap, d_len);
    return s != DET_OK ? s : t;
  } catch (...) {
    return DET_E_NOMEM;
  }
}

det_status det_host_bigint(int op, int a_sign, const uint32_t* a, int64_t alen, int b_sign,
                           const uint32_t* b, int64_t blen, int* out_sign, uint32_t* out,
                           int64_t cap, int64_t* out_len) {
  if (alen < 0 || blen < 0 || !out_len || !out_sign) return DET_E_INVALID;
  try {
    BigInt A = BigInt::from_limbs32(a, (size_t)alen, a_sign);
    BigInt B = BigInt::from_limbs32(b, (size_t)blen, b_sign);
    BigInt R, Q;
    switch (op) {
      case 0: R = A + B; break;
      case 1: R = A - B; break;
      case 2: R = A * B; break;
      case 3:
      case 4:
        if (B.sign <= 0) return DET_E_INVALID;
        BigInt::divmod_floor(A, B, Q, R);
        if (op == 3) R = Q;
        break;
      case 5: R = BigInt::gcd(A, B); break;
      default: return DET_E_INVALID;
    }
    return put(R, out_sign, out, cap, out_len);
  } catch (...) {
    return DET_E_NOMEM;
  }
}

det_status det_host_extended_bonus(const uint64_t* comb, int64_t m, int64_t k,
                                   const uint32_t* primes, int64_t np, int64_t Nbits,
                                   int64_t Dbits, uint32_t* s_mag, int64_t s_cap, int64_t* s_len,
                                   uint32_t* pi_mag, int64_t pi_cap, int64_t* pi_len,
                                   int64_t* failed) {
  if (m < 0 || m > 64 || k < 1 || np < 1 || np > 4 || !primes || Nbits < 0 || Dbits < 0 ||
      !s_len || !pi_len || !failed || (m > 0 && !comb))
    return DET_E_INVALID;
  for (int64_t z = 0; z < np; z++)
    if (primes[z] < 3) return DET_E_INVALID;
  try {
    BigInt s, pi;
    *failed = dethost::extended_bonus_host(comb, (int)m, k, primes, (int)np, Nbits, Dbits, nullptr,
                                           s, pi);
    det_status a = put(s, nullptr, s_mag, s_cap, s_len);
    det_status b = put(pi, nullptr, pi_mag, pi_cap, pi_len);
    return a != DET_OK ? a : b;
  } catch (...) {
    return DET_E_NOMEM;
  }
}

}  // extern "C"
