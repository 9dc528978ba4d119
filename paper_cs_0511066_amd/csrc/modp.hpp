// Device-side arithmetic modulo a word-size odd prime p < 2^26.
//
// Residues are kept centred, in [-(p-1)/2, (p-1)/2], stored as int32 and
// computed in FP64.  A product of two centred residues is below 2^50 in
// magnitude, so it is exact in FP64; a sum of such products stays exact as
// long as the sum of absolute values stays <= 2^53 (the chunk bound that the
// host computes and passes as `kc`).  Reduction: q = nearest integer to c / p from a
// precomputed 1/p, r = c - q p by one fused multiply-add (exact, since the
// true result is a small integer), then one fold into the centred range.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace detk {

// The integer nearest to c / p for an integer-valued |c| <= 2^53: the
// product c * (1/p) is rounded to an integer inside one fused multiply-add
// with 1.5 * 2^52 (whose unit in the last place is 1; |c / p| < 2^51), and
// the constant is taken off again.  Within one of c / p, which is all the
// reductions below need.
__device__ __forceinline__ double quot_p(double c, double pinv) {
  constexpr double RND = 6755399441055744.0;
  return fma(c, pinv, RND) - RND;
}

// c: an integer-valued double with |c| <= 2^53.  Returns c mod p, centred.
__device__ __forceinline__ double mod_c(double c, double p, double pinv) {
  double q = quot_p(c, pinv);
  double r = fma(-q, p, c);
  double h = 0.5 * p;                 // p odd: the centred range is |r| < p/2
  r = (r > h) ? r - p : r;
  r = (r < -h) ? r + p : r;
  return r;
}

// c mod p without the final fold: |c| <= 2^53 gives a result congruent to c
// with |r| <= h + 5 (h = (p-1)/2), so r == 0 exactly when p divides c.
__device__ __forceinline__ double mod_loose(double c, double p, double pinv) {
  return fma(-quot_p(c, pinv), p, c);
}

__device__ __forceinline__ double mul_mod(double a, double b, double p, double pinv) {
  return mod_c(a * b, p, pinv);
}

// Product reduced to |r| <= (p+1)/2 without the final fold: inputs with
// |a|, |b| <= (p+1)/2 keep the product below 2^52 for p < 2^26, so chains of
// these stay exact and need one fold at the end.  Four dependent operations.
__device__ __forceinline__ double mul_mod_loose(double a, double b, double p, double pinv) {
  const double c = a * b;
  return fma(-quot_p(c, pinv), p, c);
}

// a^e mod p by square-and-multiply (e >= 0); the squaring chain is the only
// dependency chain (the multiplications into r run beside it).
__device__ __forceinline__ double pow_mod(double a, uint32_t e, double p, double pinv) {
  double r = 1.0;
  double b = a;
  while (e) {
    if (e & 1u) r = mul_mod_loose(r, b, p, pinv);
    b = mul_mod_loose(b, b, p, pinv);
    e >>= 1;
  }
  return mod_c(r, p, pinv);
}

// Inverse of a non-zero residue by Fermat's little theorem, a^(p-2).
__device__ __forceinline__ double inv_mod(double a, double p, double pinv) {
  return pow_mod(a, (uint32_t)p - 2u, p, pinv);
}

// a^e mod p for e < 2^26: a fixed 26-step ladder with selects instead of
// branches (the exponent is wave-uniform).  Fully unrolled: a taken branch
// costs more than a step of the dependent chain.
__device__ __forceinline__ double pow_mod_fixed(double a, uint32_t e, double p, double pinv) {
  double r = 1.0;
  double b = a;
#pragma unroll
  for (int i = 0; i < 26; i++) {
    const double rb = mul_mod_loose(r, b, p, pinv);
    r = ((e >> i) & 1u) ? rb : r;
    b = mul_mod_loose(b, b, p, pinv);
  }
  return mod_c(r, p, pinv);
}

// Out-of-line inverse of a non-zero residue (a^(p-2)), so that call sites in
// unrolled code share one copy of the ladder.
__device__ __attribute__((noinline)) double inv_mod_call(double a, uint32_t e, double p,
                                                         double pinv) {
  return pow_mod_fixed(a, e, p, pinv);
}

// Canonical residue in [0, p) of a centred one.
__device__ __forceinline__ uint32_t to_canonical(double r, double p) {
  return (uint32_t)(int64_t)(r < 0 ? r + p : r);
}

// Per-batch-item modulus (one prime per LU in a batch).
struct Modulus {
  double p;
  double pinv;
};

}  // namespace detk
