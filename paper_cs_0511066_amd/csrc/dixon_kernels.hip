// Dixon p-adic lifting steps on gfx950 (Section 2.2: LargestInvariantFactor
// solves A x = b by p-adic lifting).  One step, with C = A^{-1} mod p:
//     x_i     = C (r_i mod p) mod p                 (k_lift_x)
//     r_{i+1} = (r_i - A x_i) / p   (exact)         (k_lift_r)
// Both are n x n matrix-vector products: one wavefront per row, lanes
// striding along the row so that every global load is coalesced.  r_i mod p
// is produced by the step that makes r_i, so it is reduced once per entry.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace detk {

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// x[row] = sum_j Cu[row][j] rp[j] mod p.  Cu, rp in [0, p), p < 2^26: each
// lane's partial sum stays below 2^64 for n <= 4096 (n/64 products < 2^52)
// and is reduced before the cross-lane sum.
__global__ __launch_bounds__(256) void k_lift_x(const uint32_t* __restrict__ Cu,
                                                const uint32_t* __restrict__ rp, int n,
                                                uint32_t p, uint32_t* __restrict__ xout) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const uint32_t* c = Cu + (int64_t)row * n;
  uint64_t acc = 0;
  for (int j = lane; j < n; j += 64) acc += (uint64_t)c[j] * rp[j];
  acc %= p;
  acc = wave_sum_u64(acc);
  if (lane == 0) xout[row] = (uint32_t)(acc % p);
}

// r[row] <- (r[row] - sum_j A[row][j] x[j]) / p and rp[row] = r[row] mod p.
// The host guarantees n ||A|| p < 2^62, so the int64 sums are exact.  The
// division is exact, so it is a multiplication by p^{-1} mod 2^64.
// Workgroup 0 also writes comb[0] = sum_j cvec[j] x[j] when comb != null
// (a random integer combination of the digit vector, for the host).
__global__ __launch_bounds__(256) void k_lift_r(const int32_t* __restrict__ Ai,
                                                const uint32_t* __restrict__ x,
                                                int64_t* __restrict__ r, uint32_t* __restrict__ rp,
                                                int n, uint32_t p, uint64_t pinv64,
                                                const uint32_t* __restrict__ cvec,
                                                uint64_t* __restrict__ comb) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row = blockIdx.x * 4 + wave;
  if (comb != nullptr && blockIdx.x == 0 && wave == 0) {
    uint64_t s = 0;
    for (int j = lane; j < n; j += 64) s += (uint64_t)cvec[j] * x[j];
    s = wave_sum_u64(s);
    if (lane == 0) comb[0] = s;
  }
  if (row >= n) return;
  const int32_t* a = Ai + (int64_t)row * n;
  int64_t acc = 0;
  for (int j = lane; j < n; j += 64) acc += (int64_t)a[j] * (int64_t)x[j];
  acc = wave_sum_i64(acc);
  if (lane == 0) {
    const int64_t t = r[row] - acc;
    const int64_t q = (int64_t)((uint64_t)t * pinv64);
    r[row] = q;
    int64_t m = q % (int64_t)p;
    if (m < 0) m += p;
    rp[row] = (uint32_t)m;
  }
}

hipError_t launch_lift_x(const uint32_t* Cu, const uint32_t* rp, int n, uint32_t p,
                         uint32_t* xout, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_lift_x<<<(n + 3) / 4, 256, 0, st>>>(Cu, rp, n, p, xout);
  return hipGetLastError();
}

hipError_t launch_lift_r(const int32_t* Ai, const uint32_t* x, int64_t* r, uint32_t* rp, int n,
                         uint32_t p, uint64_t pinv64, const uint32_t* cvec, uint64_t* comb,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_lift_r<<<(n + 3) / 4, 256, 0, st>>>(Ai, x, r, rp, n, p, pinv64, cvec, comb);
  return hipGetLastError();
}

}  // namespace detk
