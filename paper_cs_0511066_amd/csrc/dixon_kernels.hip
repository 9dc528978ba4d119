// Dixon p-adic lifting steps on gfx950 (Section 2.2: LargestInvariantFactor
// solves A x = b by p-adic lifting).  One step, with C = A^{-1} mod p:
//     x_i     = C (r_i mod p) mod p                 (phase X)
//     r_{i+1} = (r_i - A x_i) / p   (exact)         (phase R)
// Both are n x n matrix-vector products: one wavefront per row, lanes
// striding along the row with 16-byte loads.  r_i mod p is produced by the
// phase that makes r_i, so each entry is reduced once.
//
// Two launch forms: one kernel per phase (k_lift_x, k_lift_r), or, for
// n <= 1024, a single cooperative kernel that runs all k steps with the rows
// of C and A resident in registers and a grid barrier between the phases
// (k_lift_resident).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "kernels.hpp"
#include "modp.hpp"
#include "i8tile.hpp"

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

// v mod p for v < 2^64, p < 2^26: q = floor(v / p) estimated in FP64 (off by
// at most one), remainder corrected in 64-bit integer arithmetic.
__device__ __forceinline__ uint32_t umod64(uint64_t v, uint32_t p, double pinv) {
  const uint64_t q = (uint64_t)((double)v * pinv);
  int64_t r = (int64_t)(v - q * (uint64_t)p);
  r = r < 0 ? r + p : r;
  r = r >= (int64_t)p ? r - p : r;
  r = r < 0 ? r + p : r;
  r = r >= (int64_t)p ? r - p : r;
  return (uint32_t)r;
}

// v mod p in [0, p) for an integer-valued double with |v| < 2^52.
__device__ __forceinline__ double canon_p(double v, double pd, double pinv) {
  const double r = fma(-quot_p(v, pinv), pd, v);
  return r < 0.0 ? r + pd : r;
}

// v mod p in [0, p) for signed 64-bit v with |v| < 2^62.
__device__ __forceinline__ uint32_t smod64(int64_t v, uint32_t p, double pinv) {
  const int64_t q = (int64_t)floor((double)v * pinv);
  int64_t r = v - q * (int64_t)p;
  r = r < 0 ? r + p : r;
  r = r >= (int64_t)p ? r - p : r;
  r = r < 0 ? r + p : r;
  r = r >= (int64_t)p ? r - p : r;
  return (uint32_t)r;
}

// Row dot products.  Cu, rp in [0, p), p < 2^26: each lane sums at most
// n/64 products < 2^52 (below 2^58 for n <= 4096) and reduces before the
// cross-lane sum.  A: |a| < 2^31 with n ||A|| p < 2^62 (checked on the host).
// (The vector arguments carry no __restrict__: in the cooperative kernel
// they are rewritten by other workgroups between grid barriers.)
__device__ __forceinline__ uint32_t row_x(const uint32_t* __restrict__ c,
                                          const uint32_t* rp, int n, int lane,
                                          uint32_t p, double pinv) {
  uint64_t acc = 0;
  const int n4 = (n & 3) == 0 ? n : 0;      // rows are 16-byte aligned only when 4 | n
  for (int j = 4 * lane; j < n4; j += 256) {
    const uint4 cv = *(const uint4*)(c + j);
    const uint4 rv = *(const uint4*)(rp + j);
    acc += (uint64_t)cv.x * rv.x + (uint64_t)cv.y * rv.y + (uint64_t)cv.z * rv.z +
           (uint64_t)cv.w * rv.w;
  }
  for (int j = n4 + lane; j < n; j += 64) acc += (uint64_t)c[j] * rp[j];
  uint64_t s = umod64(acc, p, pinv);
  s = wave_sum_u64(s);
  return umod64(s, p, pinv);
}

__device__ __forceinline__ int64_t row_ax(const int32_t* __restrict__ a,
                                          const uint32_t* x, int n, int lane) {
  int64_t acc = 0;
  const int n4 = (n & 3) == 0 ? n : 0;
  for (int j = 4 * lane; j < n4; j += 256) {
    const int4 av = *(const int4*)(a + j);
    const uint4 xv = *(const uint4*)(x + j);
    acc += (int64_t)av.x * (int64_t)xv.x + (int64_t)av.y * (int64_t)xv.y +
           (int64_t)av.z * (int64_t)xv.z + (int64_t)av.w * (int64_t)xv.w;
  }
  for (int j = n4 + lane; j < n; j += 64) acc += (int64_t)a[j] * (int64_t)x[j];
  return wave_sum_i64(acc);
}

__device__ __forceinline__ uint64_t comb_dot(const uint32_t* __restrict__ cvec,
                                             const uint32_t* x, int n, int lane) {
  uint64_t s = 0;
  for (int j = lane; j < n; j += 64) s += (uint64_t)cvec[j] * x[j];
  return wave_sum_u64(s);
}

// r[row] <- (r[row] - dot) / p (exact: a multiplication by p^{-1} mod 2^64)
// and rp[row] = r[row] mod p.
__device__ __forceinline__ void residual_update(int64_t* __restrict__ r, uint32_t* __restrict__ rp,
                                                int row, int64_t dot, uint32_t p, double pinv,
                                                uint64_t pinv64) {
  const int64_t t = r[row] - dot;
  const int64_t q = (int64_t)((uint64_t)t * pinv64);
  r[row] = q;
  rp[row] = smod64(q, p, pinv);
}

__global__ __launch_bounds__(256) void k_lift_x(const uint32_t* __restrict__ Cu,
                                                const uint32_t* __restrict__ rp, int n,
                                                uint32_t p, double pinv,
                                                uint32_t* __restrict__ xout) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const uint32_t x = row_x(Cu + (int64_t)row * n, rp, n, lane, p, pinv);
  if (lane == 0) xout[row] = x;
}

__global__ __launch_bounds__(256) void k_lift_r(const int32_t* __restrict__ Ai,
                                                const uint32_t* __restrict__ x,
                                                int64_t* __restrict__ r, uint32_t* __restrict__ rp,
                                                int n, uint32_t p, double pinv, uint64_t pinv64,
                                                const uint32_t* __restrict__ cvec,
                                                uint64_t* __restrict__ comb) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int row = blockIdx.x * 4 + wave;
  if (comb != nullptr && blockIdx.x == 0 && wave == 0) {
    const uint64_t s = comb_dot(cvec, x, n, lane);
    if (lane == 0) comb[0] = s;
  }
  if (row >= n) return;
  const int64_t dot = row_ax(Ai + (int64_t)row * n, x, n, lane);
  if (lane == 0) residual_update(r, rp, row, dot, p, pinv, pinv64);
}

// Grid barrier of a cooperative launch: every workgroup adds one arrival to
// *bar and waits until `target` arrivals are counted.  The wait is bounded:
// after spin_limit polls the workgroup sets *err and stops waiting, and once
// *err is set no workgroup waits any more, so every wave always exits.
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned target, int* err,
                                             unsigned spin_limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    // release: this workgroup's stores (made visible to thread 0 by the
    // workgroup barrier) are published with the arrival; acquire: the
    // arrivals seen include every other workgroup's published stores.
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (++spins > spin_limit) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
}

// Loads and stores of the vectors that the three-plane lifting kernel passes
// between workgroups: device-scope relaxed atomics, served at the
// device-coherent level past the per-XCD L2 caches, so that the exchange
// needs no L2 writeback or invalidation.
__device__ __forceinline__ uint32_t ld_dev(const uint32_t* a) {
  return __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(uint32_t* a, uint32_t v) {
  __hip_atomic_store(a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Buffer resource word 3 for raw (untyped) buffer accesses on CDNA, and the
// sc1 cache-policy bit of the buffer-load builtins (device-coherent access).
constexpr int BUF_RSRC_WORD3 = 0x00020000;
constexpr int BUF_SC1 = 16;

// All k lifting steps with the rows of C and A held in registers for the
// whole loop.  Workgroups of 512 threads (8 waves, so up to 256 VGPRs per
// lane); wave w of workgroup g owns rows (8 g + w) RPW + i (i < RPW); lane l
// holds columns l + 64 e (e < EPL) of them.  Only the vectors r mod p and x_i cross the grid barriers (4n bytes
// each per phase); r itself stays in a register of lane 0.
template <int EPL, int RPW>
__global__ __launch_bounds__(512) void k_lift_resident(
    const uint32_t* __restrict__ Cu, const int32_t* __restrict__ Ai, int64_t* __restrict__ r,
    uint32_t* rp, uint32_t* xbuf, int n, uint32_t p, double pinv, uint64_t pinv64, int64_t k,
    uint32_t* __restrict__ digits, const uint32_t* __restrict__ cvec,
    uint64_t* __restrict__ comb, unsigned* bar, int* err, unsigned spin_limit) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int G = gridDim.x;
  uint32_t c[RPW][EPL];
  int32_t a[RPW][EPL];
  int64_t rr[RPW];
  int rows[RPW];
#pragma unroll
  for (int i = 0; i < RPW; i++) {
    const int row = (blockIdx.x * 8 + wave) * RPW + i;
    rows[i] = row;
    rr[i] = 0;
#pragma unroll
    for (int e = 0; e < EPL; e++) {
      const int j = lane + 64 * e;
      const bool in = row < n && j < n;
      c[i][e] = in ? Cu[(int64_t)row * n + j] : 0u;
      a[i][e] = in ? Ai[(int64_t)row * n + j] : 0;
    }
    if (row < n && lane == 0) rr[i] = r[row];
  }
  unsigned target = 0;
  for (int64_t step = 0; step < k; step++) {
    uint32_t v[EPL];
    const uint32_t* rpl = rp + lane;
#pragma unroll
    for (int e = 0; e < EPL; e++) v[e] = rpl[64 * e];
#pragma unroll
    for (int i = 0; i < RPW; i++) {
      if (rows[i] < n) {                 // wave-uniform
        uint64_t acc = 0;
#pragma unroll
        for (int e = 0; e < EPL; e++) acc += (uint64_t)c[i][e] * v[e];
        uint64_t sum = wave_sum_u64(umod64(acc, p, pinv));
        const uint32_t x = umod64(sum, p, pinv);
        if (lane == 0) {
          xbuf[rows[i]] = x;
          if (digits) digits[step * n + rows[i]] = x;
        }
      }
      __builtin_amdgcn_sched_barrier(0);   // one row at a time: bounds register pressure
    }
    target += G;
    grid_barrier(bar, target, err, spin_limit);
    const uint32_t* xl = xbuf + lane;
#pragma unroll
    for (int e = 0; e < EPL; e++) v[e] = xl[64 * e];
    if (comb != nullptr && blockIdx.x == 0 && wave == 0) {
      uint64_t sc = 0;
      const uint32_t* cl = cvec + lane;
#pragma unroll
      for (int e = 0; e < EPL; e++) sc += (uint64_t)cl[64 * e] * v[e];
      sc = wave_sum_u64(sc);
      if (lane == 0) comb[step] = sc;
    }
#pragma unroll
    for (int i = 0; i < RPW; i++) {
      if (rows[i] < n) {
        int64_t acc = 0;
#pragma unroll
        for (int e = 0; e < EPL; e++) acc += (int64_t)a[i][e] * (int64_t)v[e];
        acc = wave_sum_i64(acc);
        if (lane == 0) {
          const int64_t q = (int64_t)((uint64_t)(rr[i] - acc) * pinv64);
          rr[i] = q;
          rp[rows[i]] = smod64(q, p, pinv);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    target += G;
    grid_barrier(bar, target, err, spin_limit);
  }
#pragma unroll
  for (int i = 0; i < RPW; i++)
    if (rows[i] < n && lane == 0) r[rows[i]] = rr[i];
}

hipError_t launch_lift_x(const uint32_t* Cu, const uint32_t* rp, int n, uint32_t p,
                         uint32_t* xout, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_lift_x<<<(n + 3) / 4, 256, 0, st>>>(Cu, rp, n, p, 1.0 / (double)p, xout);
  return hipGetLastError();
}

hipError_t launch_lift_r(const int32_t* Ai, const uint32_t* x, int64_t* r, uint32_t* rp, int n,
                         uint32_t p, uint64_t pinv64, const uint32_t* cvec, uint64_t* comb,
                         hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_lift_r<<<(n + 3) / 4, 256, 0, st>>>(Ai, x, r, rp, n, p, 1.0 / (double)p, pinv64, cvec, comb);
  return hipGetLastError();
}

// Register-resident form for n <= 1024: (elements per lane, rows per wave);
// a workgroup covers 8 RPW rows.  (Larger n would not fit the registers.)
static void resident_shape(int n, int* epl, int* rpw) {
  *epl = 0;
  *rpw = 0;
  if (n <= 256) { *epl = 4; *rpw = 4; }
  else if (n <= 512) { *epl = 8; *rpw = 4; }
  else if (n <= 1024) { *epl = 16; *rpw = 2; }
}

int lift_persistent_grid(int device, int n) {
  int cus = 0, coop = 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess ||
      !coop)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  int epl, rpw;
  resident_shape(n, &epl, &rpw);
  if (epl == 0) return 0;
  const int grid = (n + 8 * rpw - 1) / (8 * rpw);
  return grid <= cus ? grid : 0;       // one workgroup per CU at most
}

// ------------------------------------------------------------------ lifting modulo p^2
// With C = A^{-1} mod p and A C = I + p E', E = E' mod p, the matrix
// C2 = C - p (C E mod p) satisfies A C2 = I (mod p^2) (one Hensel step).
// It is kept as two base-p digit planes, C2 = C + p C1 with
// C1 = (p - (C E mod p)) mod p.  Lifting modulo p^2 then yields the base-p
// digits of the solution two at a time.
//
// k_hensel<MODE>: 64x64 output tile per 256-thread workgroup, 4x4 outputs per
// thread, K in chunks of 16 through LDS, exact 64-bit accumulation.
//   MODE 0: out = ((A C - I) / p) mod p      (A int32, C in [0,p); exact since n ||A|| p < 2^62)
//   MODE 1: out = (p - (C E mod p)) mod p    (C, E in [0, p); sums below n p^2 < 2^62)
template <int MODE>
__global__ __launch_bounds__(256) void k_hensel(const void* __restrict__ Lv,
                                                const uint32_t* __restrict__ R, int n, uint32_t p,
                                                double pinv, uint64_t pinv64,
                                                uint32_t* __restrict__ out) {
  const int t = threadIdx.x;
  const int ty = t >> 4, tx = t & 15;
  const int row0 = blockIdx.y * 64, col0 = blockIdx.x * 64;
  __shared__ int64_t sL[16][65];
  __shared__ int64_t sR[16][65];
  int64_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = 0;
  for (int k0 = 0; k0 < n; k0 += 16) {
    for (int e = t; e < 64 * 16; e += 256) {
      const int r = e >> 4, kk = e & 15;
      const int gr = row0 + r, gk = k0 + kk;
      int64_t v = 0;
      if (gr < n && gk < n) {
        if (MODE == 0) v = ((const int32_t*)Lv)[(int64_t)gr * n + gk];
        else v = ((const uint32_t*)Lv)[(int64_t)gr * n + gk];
      }
      sL[kk][r] = v;
      const int kr = e >> 6, c = e & 63;
      const int gk2 = k0 + kr, gc = col0 + c;
      sR[kr][c] = (gk2 < n && gc < n) ? (int64_t)R[(int64_t)gk2 * n + gc] : 0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk++) {
      int64_t a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = sL[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = sR[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int gr = row0 + ty * 4 + i, gc = col0 + tx * 4 + j;
      if (gr >= n || gc >= n) continue;
      uint32_t v;
      if (MODE == 0) {
        const int64_t s = acc[i][j] - (gr == gc ? 1 : 0);       // divisible by p
        v = smod64((int64_t)((uint64_t)s * pinv64), p, pinv);
      } else {
        const uint32_t tt = umod64((uint64_t)acc[i][j], p, pinv);
        v = tt ? p - tt : 0u;
      }
      out[(int64_t)gr * n + gc] = v;
    }
}

// v mod P for v < 2^62, P = p^2 < 2^52 (FP64 quotient estimate, corrected).
__device__ __forceinline__ uint64_t umod_p2(uint64_t v, uint64_t P, double Pinv) {
  const uint64_t q = (uint64_t)((double)v * Pinv);
  int64_t r = (int64_t)(v - q * P);
  r = r < 0 ? r + (int64_t)P : r;
  r = r >= (int64_t)P ? r - (int64_t)P : r;
  r = r < 0 ? r + (int64_t)P : r;
  r = r >= (int64_t)P ? r - (int64_t)P : r;
  return (uint64_t)r;
}

// All lifting steps modulo p^2 with C2 = C0 + p C1 and the rows of C0, C1, A
// in registers (layout as k_lift_resident).  Vectors crossing the barriers:
// the digits (r0, r1) of r mod p^2 and (x0, x1) of x mod p^2, each padded
// with zeros.  Step s yields base-p digits 2s and 2s+1; kd digits are wanted.
template <int EPL, int RPW>
__global__ __launch_bounds__(512) void k_lift_resident2(
    const uint32_t* __restrict__ C0, const uint32_t* __restrict__ C1,
    const int32_t* __restrict__ Ai, int64_t* __restrict__ r, uint32_t* rp0, uint32_t* rp1,
    uint32_t* xb0, uint32_t* xb1, int n, uint32_t p, double pinv, uint64_t pinv64, int64_t kd,
    uint32_t* __restrict__ digits, const uint32_t* __restrict__ cvec,
    uint64_t* __restrict__ comb, unsigned* bar, int* err, unsigned spin_limit) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int G = gridDim.x;
  const uint64_t P2 = (uint64_t)p * p;
  const double P2inv = 1.0 / (double)P2;
  uint32_t c0[RPW][EPL], c1[RPW][EPL];
  int32_t a[RPW][EPL];
  int64_t rr[RPW];
  int rows[RPW];
#pragma unroll
  for (int i = 0; i < RPW; i++) {
    const int row = (blockIdx.x * 8 + wave) * RPW + i;
    rows[i] = row;
    rr[i] = 0;
#pragma unroll
    for (int e = 0; e < EPL; e++) {
      const int j = lane + 64 * e;
      const bool in = row < n && j < n;
      c0[i][e] = in ? C0[(int64_t)row * n + j] : 0u;
      c1[i][e] = in ? C1[(int64_t)row * n + j] : 0u;
      a[i][e] = in ? Ai[(int64_t)row * n + j] : 0;
    }
    if (row < n && lane == 0) rr[i] = r[row];
  }
  unsigned target = 0;
  const int64_t steps = (kd + 1) / 2;
  for (int64_t step = 0; step < steps; step++) {
    uint32_t v0[EPL], v1[EPL];
    {
      const uint32_t* l0 = rp0 + lane;
      const uint32_t* l1 = rp1 + lane;
#pragma unroll
      for (int e = 0; e < EPL; e++) {
        v0[e] = l0[64 * e];
        v1[e] = l1[64 * e];
      }
    }
#pragma unroll
    for (int i = 0; i < RPW; i++) {
      if (rows[i] < n) {
        uint64_t s0 = 0, s1 = 0;
#pragma unroll
        for (int e = 0; e < EPL; e++) {
          s0 += (uint64_t)c0[i][e] * v0[e];
          s1 += (uint64_t)c0[i][e] * v1[e] + (uint64_t)c1[i][e] * v0[e];
        }
        s0 = wave_sum_u64(umod_p2(s0, P2, P2inv));
        s1 = wave_sum_u64(umod64(s1, p, pinv));
        const uint64_t x = umod_p2(umod_p2(s0, P2, P2inv) + (uint64_t)p * umod64(s1, p, pinv), P2,
                                   P2inv);
        if (lane == 0) {
          const uint32_t xh = (uint32_t)(x / p), xl = (uint32_t)(x - (uint64_t)xh * p);
          xb0[rows[i]] = xl;
          xb1[rows[i]] = xh;
          if (digits) {
            digits[(2 * step) * n + rows[i]] = xl;
            if (2 * step + 1 < kd) digits[(2 * step + 1) * n + rows[i]] = xh;
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    target += G;
    grid_barrier(bar, target, err, spin_limit);
    {
      const uint32_t* l0 = xb0 + lane;
      const uint32_t* l1 = xb1 + lane;
#pragma unroll
      for (int e = 0; e < EPL; e++) {
        v0[e] = l0[64 * e];
        v1[e] = l1[64 * e];
      }
    }
    if (comb != nullptr && blockIdx.x == 0 && wave == 0) {
      uint64_t s0 = 0, s1 = 0;
      const uint32_t* cl = cvec + lane;
#pragma unroll
      for (int e = 0; e < EPL; e++) {
        s0 += (uint64_t)cl[64 * e] * v0[e];
        s1 += (uint64_t)cl[64 * e] * v1[e];
      }
      s0 = wave_sum_u64(s0);
      s1 = wave_sum_u64(s1);
      if (lane == 0) {
        comb[2 * step] = s0;
        if (2 * step + 1 < kd) comb[2 * step + 1] = s1;
      }
    }
#pragma unroll
    for (int i = 0; i < RPW; i++) {
      if (rows[i] < n) {
        int64_t d0 = 0, d1 = 0;
#pragma unroll
        for (int e = 0; e < EPL; e++) {
          d0 += (int64_t)a[i][e] * (int64_t)v0[e];
          d1 += (int64_t)a[i][e] * (int64_t)v1[e];
        }
        d0 = wave_sum_i64(d0);
        d1 = wave_sum_i64(d1);
        if (lane == 0) {
          // r' = ((r - A x0)/p - A x1)/p, both divisions exact
          const int64_t t1 = (int64_t)((uint64_t)(rr[i] - d0) * pinv64);
          const int64_t q = (int64_t)((uint64_t)(t1 - d1) * pinv64);
          rr[i] = q;
          const uint32_t m0 = smod64(q, p, pinv);
          const int64_t qd = (int64_t)((uint64_t)(q - (int64_t)m0) * pinv64);   // (q - m0)/p
          rp0[rows[i]] = m0;
          rp1[rows[i]] = smod64(qd, p, pinv);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    target += G;
    grid_barrier(bar, target, err, spin_limit);
  }
#pragma unroll
  for (int i = 0; i < RPW; i++)
    if (rows[i] < n && lane == 0) r[rows[i]] = rr[i];
}

hipError_t launch_hensel(const int32_t* Ai, const uint32_t* Cu, uint32_t* E, uint32_t* C1, int n,
                         uint32_t p, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid((n + 63) / 64, (n + 63) / 64);
  uint64_t pinv64 = (uint64_t)p;
  for (int i = 0; i < 5; i++) pinv64 *= 2 - (uint64_t)p * pinv64;
  const double pinv = 1.0 / (double)p;
  k_hensel<0><<<grid, 256, 0, st>>>((const void*)Ai, Cu, n, p, pinv, pinv64, E);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_hensel<1><<<grid, 256, 0, st>>>((const void*)Cu, E, n, p, pinv, pinv64, C1);
  return hipGetLastError();
}

hipError_t launch_lift_resident2(int grid, const uint32_t* C0, const uint32_t* C1,
                                 const int32_t* Ai, int64_t* r, uint32_t* rp0, uint32_t* rp1,
                                 uint32_t* xb0, uint32_t* xb1, int n, uint32_t p, uint64_t pinv64,
                                 int64_t kd, uint32_t* digits, const uint32_t* cvec,
                                 uint64_t* comb, unsigned* bar, int* err, hipStream_t st) {
  if (n <= 0 || kd <= 0) return hipSuccess;
  double pinv = 1.0 / (double)p;
  unsigned spin_limit = 1u << 22;     // ~0.1 s of polling per barrier at most
  void* args[] = {(void*)&C0, (void*)&C1, (void*)&Ai, (void*)&r, (void*)&rp0, (void*)&rp1,
                  (void*)&xb0, (void*)&xb1, (void*)&n, (void*)&p, (void*)&pinv, (void*)&pinv64,
                  (void*)&kd, (void*)&digits, (void*)&cvec, (void*)&comb, (void*)&bar,
                  (void*)&err, (void*)&spin_limit};
  int epl, rpw;
  resident_shape(n, &epl, &rpw);
  const void* f = nullptr;
  if (epl == 4) f = (const void*)k_lift_resident2<4, 4>;
  else if (epl == 8) f = (const void*)k_lift_resident2<8, 4>;
  else if (epl == 16) f = (const void*)k_lift_resident2<16, 2>;
  if (!f || grid != (n + 8 * rpw - 1) / (8 * rpw)) return hipErrorInvalidValue;
  return hipLaunchCooperativeKernel(f, dim3(grid), dim3(512), args, 0, st);
}

// Shape of the three-plane kernel: 8 waves per workgroup, 2 rows per wave.
// Shape of the three-plane lifting: LIFT3_NWAVE waves of LIFT3_RPW rows per
// workgroup, one workgroup per LIFT3_RPW * LIFT3_NWAVE rows.
constexpr int LIFT3_RPW = 1, LIFT3_NWAVE = 8;
static int lift3_grid_size(int n) {
  return (n + LIFT3_RPW * LIFT3_NWAVE - 1) / (LIFT3_RPW * LIFT3_NWAVE);
}

int lift3_max_rhs(int n) { return n <= 1024 ? LIFT3_MAX_RHS : 1; }

// Liftings side by side in one launch: the forms up to order 1024 (planes and
// A as FP64 registers, one workgroup a CU) take LIFT_MAX_PRIMES x their grid
// at most; the narrow forms above it take one.
static int lift3_max_primes_of(int n) { return n <= 1024 ? LIFT_MAX_PRIMES : 1; }

int lift3_max_primes(int device, int n) {
  const int grid = lift3_grid(device, n);
  int cus = 0;
  if (grid <= 0 ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  return std::max(1, std::min(lift3_max_primes_of(n), cus / grid));
}

int lift3_grid(int device, int n) {
  int cus = 0, coop = 0;
  if (n > 2048) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess ||
      !coop)
    return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return 0;
  const int grid = lift3_grid_size(n);
  return grid <= cus ? grid : 0;
}

// ------------------------------------------------------------------ lifting modulo p^3 in FP64
// For p < 2^25 and n ||A|| p < 2^53 every product and partial sum below is an
// integer of magnitude < 2^53, so FP64 arithmetic is exact and runs at the
// full vector rate (64-bit integer multiplies run at a quarter of it).
//
// Hensel planes of C = A^{-1} mod p^3, C = c0 + p c1 + p^2 c2, by the
// linear Hensel recursion with full integer error matrices:
//   E_1 = (A c0 - I) / p,  C_k = -c0 E_k mod p,  E_{k+1} = (E_k + A c_k) / p,
// where c_k is the centred representative of the stored plane C_k in [0, p)
// (A C^{(k)} = I + p^k E_k exactly, and E_k + A c_k = 0 mod p).  The lifting
// kernel uses the same centred representatives.
//
// k_hensel_f64<MODE>: a 64x64 output tile per 256-thread workgroup on FP64
// MFMA (v_mfma_f64_16x16x4f64; each wave a 32x32 quarter as 2x2 blocks),
// K in chunks of 64 through LDS; the next chunk's global loads are issued
// before the current chunk's 64 MFMAs a wave, so their latency is hidden.
//   MODE 0: Eout = (Ein + A c_k) / p   (Ein = -I when Ein == null).  Every
//           partial sum is below n ||A|| p / 2 < 2^53: exact without reduction;
//           the quotient is exact, so rint of the scaled sum is it.
//   MODE 1: Cout = (-c0 E) mod p in [0, p), E reduced to centred residues on
//           load; products < 2^48 (p < 2^25), reduced every 16 k-steps.
typedef double v4d_h __attribute__((ext_vector_type(4)));
template <int MODE>
__global__ __launch_bounds__(512) void k_hensel_f64(const void* __restrict__ Lv0,
                                                    const void* __restrict__ Rv0,
                                                    const double* __restrict__ Ein0, int n,
                                                    PrimeSet ps, int64_t sLz, int64_t sRz,
                                                    int64_t sEz, void* __restrict__ out0) {
  constexpr int BM = 64, BN = 64, BK = 64;
  constexpr int T = 512;                                    // eight waves of 32 x 16
  constexpr int NL = BM * BK / T, NR = BK * BN / T;         // values a thread loads per chunk
  typedef typename std::conditional<MODE == 0, uint32_t, double>::type rv_t;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;
  const int row0 = blockIdx.y * BM, col0 = blockIdx.x * BN;
  // prime z of the batch: its operands at element offsets z sLz, z sRz, z sEz
  // (an offset of 0 shares the operand), its output at z n^2
  const int z = blockIdx.z;
  const uint32_t p = ps.p[z];
  const double pinv = ps.pinv[z];
  typedef typename std::conditional<MODE == 0, uint32_t, double>::type rv0_t;
  typedef typename std::conditional<MODE == 0, double, uint32_t>::type out_t;
  const void* Lv = (const uint32_t*)Lv0 + (int64_t)z * sLz;
  const void* Rv = (const rv0_t*)Rv0 + (int64_t)z * sRz;
  const double* Ein = Ein0 ? Ein0 + (int64_t)z * sEz : nullptr;
  void* out = (out_t*)out0 + (int64_t)z * n * n;
  const double pd = (double)p, h = 0.5 * pd;
  __shared__ double sL[BK][BM + 2];
  __shared__ double sR[BK][BN + 2];
  // chunk loads, consecutive threads on consecutive addresses: value u of
  // thread t is element u * 256 + t of the tile in row-major order
  uint32_t lreg[NL];
  rv_t rreg[NR];
  // (unconditional loads from clamped indices: a load under a condition
  // waits for its own data; entries outside A are zeroed at the store)
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int f = u * T + t, r = f / BK, k = f % BK;
      lreg[u] = ((const uint32_t*)Lv)[(int64_t)min(row0 + r, n - 1) * n + min(k0 + k, n - 1)];
    }
#pragma unroll
    for (int u = 0; u < NR; u++) {
      const int f = u * T + t, k = f / BN, c = f % BN;
      rreg[u] = ((const rv_t*)Rv)[(int64_t)min(k0 + k, n - 1) * n + min(col0 + c, n - 1)];
    }
  };
  // to LDS as FP64: A as int32; planes centred; E reduced
  auto lstore = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int f = u * T + t, r = f / BK, k = f % BK;
      double v;
      if (MODE == 0) {
        v = (double)(int32_t)lreg[u];
      } else {
        const double w = (double)lreg[u];
        v = w > h ? w - pd : w;
      }
      sL[k][r] = (row0 + r < n && k0 + k < n) ? v : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NR; u++) {
      const int f = u * T + t, k = f / BN, c = f % BN;
      double v;
      if (MODE == 0) {
        const double w = (double)rreg[u];
        v = w > h ? w - pd : w;
      } else {
        v = mod_c((double)rreg[u], pd, pinv);
      }
      sR[k][c] = (k0 + k < n && col0 + c < n) ? v : 0.0;
    }
  };
  v4d_h acc[2][1];
#pragma unroll
  for (int i = 0; i < 2; i++) acc[i][0] = (v4d_h){0.0, 0.0, 0.0, 0.0};
  gload(0);
  for (int k0 = 0; k0 < n; k0 += BK) {
    lstore(k0);
    __syncthreads();
    if (k0 + BK < n) gload(k0 + BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[2];
#pragma unroll
      for (int i = 0; i < 2; i++) af[i] = sL[kr][wr * 32 + i * 16 + (lane & 15)];
      const double bf = sR[kr][wc * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; i++)
        acc[i][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf, acc[i][0], 0, 0, 0);
      if (MODE == 1 && (ks & 15) == 12) {
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int r = 0; r < 4; r++) acc[i][0][r] = mod_loose(acc[i][0][r], pd, pinv);
      }
    }
    __syncthreads();
  }
  // output element (row wr*32 + i*16 + lane/16 + 4 r, col wc*16 + lane%16);
  // MODE 0 reads Ein for all of them first (clamped, unconditional)
  const int gc = col0 + wc * 16 + (lane & 15);
  double ein[2][4];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int gr = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
      ein[i][r] = (MODE == 0 && Ein) ? Ein[(int64_t)min(gr, n - 1) * n + min(gc, n - 1)]
                                     : (gr == gc ? -1.0 : 0.0);
    }
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int gr = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
      if (gr >= n || gc >= n) continue;
      const int64_t o = (int64_t)gr * n + gc;
      if (MODE == 0) {
        ((double*)out)[o] = quot_p(ein[i][r] + acc[i][0][r], pinv);
      } else {
        const double v = mod_c(-acc[i][0][r], pd, pinv);
        ((uint32_t*)out)[o] = (uint32_t)(v < 0 ? v + pd : v);
      }
    }
}

// ------------------------------------------------------------------ Hensel products on int8 MFMA
// The same four products as k_hensel_f64, on three signed int8 limbs of each
// operand (i8tile.hpp) with int32 accumulation: every operand value lies in
// [-LIMB3_MAX, LIMB3_MAX] (entries of A, and centred residues for p <=
// 2 LIMB3_MAX + 1), so the limb products give the exact integer product.
// k_split_h<SRC>: limb planes of prime z's n x n operand (transposed for the
// right-hand factor), SRC 0: int32 values taken as they are (A, shared: sz =
// 0); 1: canonical residues in [0, p), centred; 2: FP64 integers (E),
// reduced mod p and centred.
template <int SRC>
__global__ __launch_bounds__(256) void k_split_h(const void* __restrict__ src, int64_t sz, int n,
                                                 int Kp, int64_t Rp, int transpose,
                                                 int8_t* __restrict__ P, int64_t pslab,
                                                 PrimeSet ps) {
  __shared__ uint32_t sT[64][65];
  const int z = blockIdx.z;
  const uint32_t p = ps.p[z];
  const double pd = (double)p, pinv = ps.pinv[z];
  auto get = [&](int r, int c) -> int32_t {
    const int64_t o = (int64_t)z * sz + (int64_t)r * n + c;
    if (SRC == 0) return ((const int32_t*)src)[o];
    if (SRC == 1) {
      const uint32_t u = ((const uint32_t*)src)[o];
      return u > (p - 1) / 2 ? (int32_t)u - (int32_t)p : (int32_t)u;
    }
    return (int32_t)mod_c(((const double*)src)[o], pd, pinv);
  };
  limb_split_tile(get, n, n, Kp, Rp, transpose, P + (int64_t)z * pslab, sT);
}

// k_hensel_i8<MODE>: the 64 x 64 output tile of prime z from the limb planes
// (PA: left factor, PB: right factor transposed; Rp x Kp a plane).  With v
// the exact product (the limb sums weighted by 2^(8s), in int64):
//   MODE 0: E = (Ein + v) / p (Ein = -I when null), exact in FP64 (|Ein + v|
//           < 2^53 under the lifting's bound), as k_hensel_f64;
//   MODE 1: C = -v mod p in [0, p).
template <int MODE>
__global__ __launch_bounds__(256) void k_hensel_i8(const int8_t* __restrict__ PA,
                                                   const int8_t* __restrict__ PB,
                                                   int64_t pslabA, int64_t pslabB, int64_t Rp,
                                                   int Kp, int n, PrimeSet ps,
                                                   const double* __restrict__ Ein, int64_t sE,
                                                   void* __restrict__ out0) {
  const int z = blockIdx.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const uint32_t p = ps.p[z];
  const double pd = (double)p, pinv = ps.pinv[z];
  const int row0 = blockIdx.y * I8_TILE, col0 = blockIdx.x * I8_TILE;
  __shared__ __attribute__((aligned(16))) int8_t sA[3][I8_TILE][I8_LD];
  __shared__ __attribute__((aligned(16))) int8_t sB[3][I8_TILE][I8_LD];
  v4i_t acc[5][2][2];
  i8_tile_product(PA + (int64_t)z * pslabA, PB + (int64_t)z * pslabB, Rp * Kp, Rp * Kp, Kp, row0,
                  col0, sA, sB, acc);
  const int64_t nn = (int64_t)n * n;
  double wgt[5];                                    // 2^(8s) mod p, centred (MODE 1)
  wgt[0] = 1.0;
#pragma unroll
  for (int s = 1; s < 5; s++) wgt[s] = mod_c(wgt[s - 1] * 256.0, pd, pinv);
  // MODE 0 reads Ein for all its elements first (clamped, unconditional)
  double ein[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int gr = row0 + wr * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int gc = col0 + wc * 32 + j * 16 + (lane & 15);
        ein[i][j][r] = (MODE == 0 && Ein)
                           ? Ein[(int64_t)z * sE + (int64_t)min(gr, n - 1) * n + min(gc, n - 1)]
                           : (gr == gc ? -1.0 : 0.0);
      }
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int gr = row0 + wr * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int gc = col0 + wc * 32 + j * 16 + (lane & 15);
        if (gr >= n || gc >= n) continue;
        const int64_t o = (int64_t)z * nn + (int64_t)gr * n + gc;
        if (MODE == 0) {
          int64_t v = 0;
#pragma unroll
          for (int s = 4; s >= 0; s--) v = v * 256 + (int64_t)acc[s][i][j][r];
          ((double*)out0)[o] = quot_p(ein[i][j][r] + (double)v, pinv);
        } else {
          double v = 0.0;
#pragma unroll
          for (int s = 0; s < 5; s++) v += mod_c((double)acc[s][i][j][r], pd, pinv) * wgt[s];
          v = mod_c(-v, pd, pinv);
          ((uint32_t*)out0)[o] = (uint32_t)(v < 0 ? v + pd : v);
        }
      }
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Wave sums through DPP row operations (quad permutes, row rotations, row
// broadcasts): six VALU steps instead of six LDS round trips; the total is
// read from lane 63 and is the same in every lane afterwards.
__device__ __forceinline__ int dpp_sum_i32(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);    // quad_perm [1,0,3,2]
  x += __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);    // quad_perm [2,3,0,1]
  x += __builtin_amdgcn_update_dpp(0, x, 0x124, 0xF, 0xF, false);   // row_ror:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);   // row_ror:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);   // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);   // row_bcast:31
  return __builtin_amdgcn_readlane(x, 63);
}

template <int CTRL, int RMASK>
__device__ __forceinline__ double dpp_mov_f64(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, RMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, RMASK, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// Exact when every partial sum is an integer below 2^53 in magnitude.
__device__ __forceinline__ double dpp_sum_f64(double x) {
  x += dpp_mov_f64<0xB1, 0xF>(x);
  x += dpp_mov_f64<0x4E, 0xF>(x);
  x += dpp_mov_f64<0x124, 0xF>(x);
  x += dpp_mov_f64<0x128, 0xF>(x);
  x += dpp_mov_f64<0x142, 0xA>(x);
  x += dpp_mov_f64<0x143, 0xC>(x);
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ int32_t centred_i32(uint32_t u, uint32_t p) {
  return u > (p - 1) / 2 ? (int32_t)u - (int32_t)p : (int32_t)u;
}

// All lifting steps modulo p^3 in FP64, three base-p digits per step, with
// the centred planes c0, c1, c2 of A^{-1} mod p^3 and the rows of A in
// registers (c0, c1 as FP64; c2 and A as FP64, or as int32 converted at their
// use when NARROW): wave w of workgroup g (NWAVE waves, RG = RPW NWAVE
// rows) owns rows g RG + w RPW + i (i < RPW), lane l columns l + 64 e
// (e < EPL).  Vectors passed between workgroups: the three digits of r mod
// p^3, balanced (|digit| <= (p-1)/2, r = w0 + p w1 + p^2 w2 mod p^3), and the
// three digits of x in [0, p), row by row in 16 bytes per right-hand side
// (rv, xv: n x NRHS x 4 words, the fourth word holding only the tag; NRHS
// right-hand sides share the planes, the rows of A and the exchanges).
// Phase X, per lane over its EPL columns (w_q = centred digit q of r):
//   S0 = sum c0 w0, S1 = sum c0 w1 + c1 w0, S2 = sum c0 w2 + c1 w1 + c2 w0,
// each partial sum of 16 products below 2^52; carries are taken lane by lane
// (S0 = q0 p + m0, ...), so the three lane digits m0, m1, m2 are small and
// their wave sums fit in int32; digits of x follow with a carry pass.
// Phase R: D_q = A x_q (|D_q| <= n ||A|| p < 2^53) and
//   r' = (((r - D0)/p - D1)/p - D2)/p,
// every partial value an integer below 2^53 (|r| stays below n ||A|| + ||b||),
// so the per-row steps run in FP64 too: an exact quotient by p is
// the integer nearest to v * (1/p) (quot_p), as |v / p| < 2^28 keeps the
// error of the reciprocal far below 1/2.
//
// No grid barrier: every exchanged 32-bit word holds a 25-bit digit (two's
// complement for r, plain for x) under a 7-bit tag, the step number mod 127,
// and is written and read at the device-coherent level; a reader polls until
// the words it wants carry the tag of its step.  The words of x of step s are
// written only after their writer has read all of r of step s, and each word
// of r of step s+1 only after its writer has read all of x of step s, so a
// word is never overwritten before every workgroup has read it, and a reader
// finds in it either the value it waits for or the one before it (another
// tag).  Tags run over 0..126: the caller fills xv with all-ones words (tag
// 127) before the launch and writes r of step 0 with tag 0.  Each workgroup
// gathers its rows in LDS and writes them with one store instruction: many
// small writes into one segment, one per digit and row, take several times
// longer to become visible than one contiguous write.  A wait that exceeds
// spin_limit polls sets *err; after that every wait gives up within 64
// polls, so all waves exit.
template <int EPL, int RPW, int NWAVE, int NRHS, bool NARROW>
__global__ __launch_bounds__(64 * NWAVE) void k_lift_resident3(
    const uint32_t* __restrict__ C0g, const uint32_t* __restrict__ C1g,
    const uint32_t* __restrict__ C2g, const int32_t* __restrict__ Ai, int64_t* __restrict__ rg,
    uint32_t* rvg, uint32_t* xvg, int n, PrimeSet ps, int gpp, int64_t kd,
    uint32_t* __restrict__ digitsg, int64_t dig_rhs_stride, int64_t dig_prime_stride, int* err,
    unsigned spin_limit) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // the lifting of prime z runs on workgroups [z gpp, (z + 1) gpp), on its
  // own planes, vectors and digits (the rows of A are shared)
  const int z = blockIdx.x / gpp;
  const int blk = blockIdx.x - z * gpp;
  const uint32_t p = ps.p[z];
  const double pinv = ps.pinv[z];
  const int64_t nn = (int64_t)n * n;
  const uint32_t* __restrict__ C0 = C0g + z * nn;
  const uint32_t* __restrict__ C1 = C1g + z * nn;
  const uint32_t* __restrict__ C2 = C2g + z * nn;
  int64_t* __restrict__ r = rg + (int64_t)z * n * NRHS;
  uint32_t* rv = rvg + (int64_t)z * n * NRHS * 4;
  uint32_t* xv = xvg + (int64_t)z * n * NRHS * 4;
  uint32_t* __restrict__ digits = digitsg ? digitsg + z * dig_prime_stride : nullptr;
  const double pd = (double)p;
  constexpr uint32_t DIG = LIFT3_DIGIT_MASK;
  constexpr int RG = RPW * NWAVE;                       // rows per workgroup
  constexpr int NC = 64 * EPL;                          // columns (at least n)
  constexpr int NJ = (EPL + NWAVE - 1) / NWAVE;         // rows staged per thread
  const int row0 = blk * RG;
  // the vectors a phase reads, staged once per workgroup as int32 (digit t of
  // row j for right-hand side h at [h][t][j]: every wave reads all of it), one
  // buffer per phase so that a phase may stage while slower waves still read
  // the other phase's buffer
  __shared__ int32_t sV[2][NRHS][3][NC];
  // the workgroup's records of the vectors a phase writes, gathered for one store
  __shared__ uint32_t sOut[RG * NRHS * 4];
  // 16-byte loads at the device-coherent level: buffer loads with the sc1
  // cache policy (offsets past the vectors read as zero)
  const int nbytes = 16 * n * NRHS;
  const __amdgpu_buffer_rsrc_t rsr = __builtin_amdgcn_make_buffer_rsrc(rv, 0, nbytes, BUF_RSRC_WORD3);
  const __amdgpu_buffer_rsrc_t rsx = __builtin_amdgcn_make_buffer_rsrc(xv, 0, nbytes, BUF_RSRC_WORD3);
  bool gave_up = false;
  // Staging of one set of vectors: every thread reads the records of its NJ
  // rows and polls again those whose tag is still old; after spin_limit polls
  // it sets *err (or gives up on finding it set).
  auto stage3 = [&](int32_t (*s)[3][NC], __amdgpu_buffer_rsrc_t src, uint32_t tag, bool sgn) {
    u32x4 a[NJ][NRHS];
    bool want[NJ][NRHS];
#pragma unroll
    for (int q = 0; q < NJ; q++) {
      const int j = threadIdx.x + 64 * NWAVE * q;
#pragma unroll
      for (int h = 0; h < NRHS; h++) {
        want[q][h] = j < n && j < NC;
        a[q][h] = u32x4{0, 0, 0, 0};
      }
    }
    unsigned spins = 0;
    for (;;) {
      // every record is read on every poll (a load under a condition would
      // wait for its data before the next is issued; offsets past the
      // vectors read as zero), and only the rows still wanted take the value
      u32x4 b[NJ][NRHS];
#pragma unroll
      for (int q = 0; q < NJ; q++)
#pragma unroll
        for (int h = 0; h < NRHS; h++) {
          int off = 16 * ((threadIdx.x + 64 * NWAVE * q) * NRHS + h);
          asm volatile("" : "+v"(off));      // a fresh load on every poll
          b[q][h] = __builtin_amdgcn_raw_buffer_load_b128(src, off, 0, BUF_SC1);
        }
#pragma unroll
      for (int q = 0; q < NJ; q++)
#pragma unroll
        for (int h = 0; h < NRHS; h++)
          if (want[q][h]) a[q][h] = b[q][h];
      bool pending = false;
#pragma unroll
      for (int q = 0; q < NJ; q++)
#pragma unroll
        for (int h = 0; h < NRHS; h++) {
          if (want[q][h] && (a[q][h].x >> 25) == tag && (a[q][h].y >> 25) == tag &&
              (a[q][h].z >> 25) == tag)
            want[q][h] = false;
          pending |= want[q][h];
        }
      if (!pending || gave_up) break;
      if ((++spins & 63) == 0) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
          gave_up = true;
          break;
        }
        if (spins > spin_limit) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          gave_up = true;
          break;
        }
      }
      __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int q = 0; q < NJ; q++) {
      const int j = threadIdx.x + 64 * NWAVE * q;
      if (j < NC) {
#pragma unroll
        for (int h = 0; h < NRHS; h++) {
          // r digits: sign-extend the 25-bit field; x digits: the field itself
          s[h][0][j] = sgn ? (int32_t)(a[q][h].x << 7) >> 7 : (int32_t)(a[q][h].x & DIG);
          s[h][1][j] = sgn ? (int32_t)(a[q][h].y << 7) >> 7 : (int32_t)(a[q][h].y & DIG);
          s[h][2][j] = sgn ? (int32_t)(a[q][h].z << 7) >> 7 : (int32_t)(a[q][h].z & DIG);
        }
      }
    }
    __syncthreads();
  };
  // the workgroup writes its gathered records: one word per thread
  auto publish = [&](uint32_t* v) {
    __syncthreads();
    if (threadIdx.x < 4 * RG * NRHS && row0 + (int)threadIdx.x / (4 * NRHS) < n)
      st_dev(v + (size_t)row0 * NRHS * 4 + threadIdx.x, sOut[threadIdx.x]);
  };
  // centred planes and the rows of A in registers: c0, c1 as FP64; c2 and A
  // as FP64, or (NARROW, for the largest orders) as int32 converted at use
  typedef typename std::conditional<NARROW, int32_t, double>::type nar_t;
  double c0[RPW][EPL], c1[RPW][EPL];
  nar_t c2[RPW][EPL], av[RPW][EPL];
  double rr[RPW][NRHS];                            // r of the row (lane 0), integers
  int rows[RPW];
#pragma unroll
  for (int i = 0; i < RPW; i++) {
    const int row = row0 + wave * RPW + i;
    rows[i] = row;
    // the row's loads four entries a plane at a time, all in flight
    // together, from clamped indices (a load under a condition waits for its
    // own data); entries outside A are zero
    static_assert(EPL % 4 == 0, "entries per lane");
#pragma unroll
    for (int e0 = 0; e0 < EPL; e0 += 4) {
      uint32_t l0[4], l1[4], l2[4];
      int32_t la[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int64_t o = (int64_t)min(row, n - 1) * n + min(lane + 64 * (e0 + u), n - 1);
        l0[u] = C0[o];
        l1[u] = C1[o];
        l2[u] = C2[o];
        la[u] = Ai[o];
      }
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int e = e0 + u;
        const bool in = row < n && lane + 64 * e < n;
        c0[i][e] = in ? (double)centred_i32(l0[u], p) : 0.0;
        c1[i][e] = in ? (double)centred_i32(l1[u], p) : 0.0;
        c2[i][e] = in ? (nar_t)centred_i32(l2[u], p) : (nar_t)0;
        av[i][e] = in ? (nar_t)la[u] : (nar_t)0;
      }
    }
#pragma unroll
    for (int h = 0; h < NRHS; h++)
      rr[i][h] = (row < n && lane == 0) ? (double)r[(int64_t)row * NRHS + h] : 0.0;
  }
  const int64_t steps = (kd + 2) / 3;
  uint32_t tag = 0;                                // step mod 127
  for (int64_t step = 0; step < steps; step++) {
    const uint32_t tag1 = tag == 126 ? 0 : tag + 1;
    // ---- phase X
    double S0[RPW][NRHS], S1a[RPW][NRHS], S1b[RPW][NRHS], S2a[RPW][NRHS], S2b[RPW][NRHS],
        S2c[RPW][NRHS];
#pragma unroll
    for (int i = 0; i < RPW; i++)
#pragma unroll
      for (int h = 0; h < NRHS; h++)
        S0[i][h] = S1a[i][h] = S1b[i][h] = S2a[i][h] = S2b[i][h] = S2c[i][h] = 0.0;
    stage3(sV[0], rsr, tag, true);
#pragma unroll
    for (int e = 0; e < EPL; e++) {
#pragma unroll
      for (int h = 0; h < NRHS; h++) {
        const double w0 = (double)sV[0][h][0][lane + 64 * e];    // balanced digits
        const double w1 = (double)sV[0][h][1][lane + 64 * e];
        const double w2 = (double)sV[0][h][2][lane + 64 * e];
#pragma unroll
        for (int i = 0; i < RPW; i++) {
          S0[i][h] = fma(c0[i][e], w0, S0[i][h]);
          S1a[i][h] = fma(c0[i][e], w1, S1a[i][h]);
          S1b[i][h] = fma(c1[i][e], w0, S1b[i][h]);
          S2a[i][h] = fma(c0[i][e], w2, S2a[i][h]);
          S2b[i][h] = fma(c1[i][e], w1, S2b[i][h]);
          S2c[i][h] = fma((double)c2[i][e], w0, S2c[i][h]);
        }
      }
    }
    // (absent rows, whose planes are 0, run through as well)
#pragma unroll
    for (int i = 0; i < RPW; i++)
#pragma unroll
      for (int h = 0; h < NRHS; h++) {
        const double q0 = quot_p(S0[i][h], pinv), m0 = fma(-q0, pd, S0[i][h]);
        const double qa = quot_p(S1a[i][h], pinv), ma = fma(-qa, pd, S1a[i][h]);
        const double T1 = ma + S1b[i][h] + q0;
        const double q1 = quot_p(T1, pinv), m1 = fma(-q1, pd, T1);
        const double T2 = mod_loose(S2a[i][h], pd, pinv) + mod_loose(S2b[i][h], pd, pinv) +
                          mod_loose(S2c[i][h], pd, pinv) + qa + q1;
        const double m2 = mod_loose(T2, pd, pinv);
        const int64_t M0 = dpp_sum_i32((int)m0);
        const int64_t M1 = dpp_sum_i32((int)m1);
        const int64_t M2 = dpp_sum_i32((int)m2);
        if (rows[i] < n && lane == 0) {
          // carries (|M| < 2^31): exact quotients by p in FP64
          const double x0d = canon_p((double)M0, pd, pinv);
          const double t1 = (double)M1 + quot_p((double)M0 - x0d, pinv);
          const double x1d = canon_p(t1, pd, pinv);
          const double t2 = (double)M2 + quot_p(t1 - x1d, pinv);
          const uint32_t x0 = (uint32_t)x0d, x1 = (uint32_t)x1d;
          const uint32_t x2 = (uint32_t)canon_p(t2, pd, pinv);
          uint32_t* o = sOut + ((wave * RPW + i) * NRHS + h) * 4;
          o[0] = tag << 25 | x0;
          o[1] = tag << 25 | x1;
          o[2] = tag << 25 | x2;
          o[3] = tag << 25;
          if (digits) {
            uint32_t* dg = digits + (int64_t)h * dig_rhs_stride;
            dg[(3 * step) * n + rows[i]] = x0;
            if (3 * step + 1 < kd) dg[(3 * step + 1) * n + rows[i]] = x1;
            if (3 * step + 2 < kd) dg[(3 * step + 2) * n + rows[i]] = x2;
          }
        }
      }
    publish(xv);
    // ---- phase R
    double D0[RPW][NRHS], D1[RPW][NRHS], D2[RPW][NRHS];
#pragma unroll
    for (int i = 0; i < RPW; i++)
#pragma unroll
      for (int h = 0; h < NRHS; h++) D0[i][h] = D1[i][h] = D2[i][h] = 0.0;
    stage3(sV[1], rsx, tag, false);
#pragma unroll
    for (int e = 0; e < EPL; e++) {
#pragma unroll
      for (int h = 0; h < NRHS; h++) {
        const double x0 = (double)sV[1][h][0][lane + 64 * e];
        const double x1 = (double)sV[1][h][1][lane + 64 * e];
        const double x2 = (double)sV[1][h][2][lane + 64 * e];
#pragma unroll
        for (int i = 0; i < RPW; i++) {
          const double ae = (double)av[i][e];
          D0[i][h] = fma(ae, x0, D0[i][h]);
          D1[i][h] = fma(ae, x1, D1[i][h]);
          D2[i][h] = fma(ae, x2, D2[i][h]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RPW; i++)
#pragma unroll
      for (int h = 0; h < NRHS; h++) {
        const double d0 = dpp_sum_f64(D0[i][h]);
        const double d1 = dpp_sum_f64(D1[i][h]);
        const double d2 = dpp_sum_f64(D2[i][h]);
        if (rows[i] < n && lane == 0) {
          // exact divisions by p
          double q = quot_p(rr[i][h] - d0, pinv);
          q = quot_p(q - d1, pinv);
          q = quot_p(q - d2, pinv);
          rr[i][h] = q;
          // balanced digits of r' mod p^3, the carry of each centring taken
          // into the next digit, so that m0 + p m1 + p^2 m2 = r' (mod p^3)
          const double m0d = mod_c(q, pd, pinv);
          const double u1 = quot_p(q - m0d, pinv);
          const double m1d = mod_c(u1, pd, pinv);
          const double u2 = quot_p(u1 - m1d, pinv);
          const int32_t m0 = (int32_t)m0d, m1 = (int32_t)m1d;
          const int32_t m2 = (int32_t)mod_c(u2, pd, pinv);
          uint32_t* o = sOut + ((wave * RPW + i) * NRHS + h) * 4;
          o[0] = tag1 << 25 | ((uint32_t)m0 & DIG);
          o[1] = tag1 << 25 | ((uint32_t)m1 & DIG);
          o[2] = tag1 << 25 | ((uint32_t)m2 & DIG);
          o[3] = tag1 << 25;
        }
      }
    publish(rv);
    tag = tag1;
  }
#pragma unroll
  for (int i = 0; i < RPW; i++)
#pragma unroll
    for (int h = 0; h < NRHS; h++)
      if (rows[i] < n && lane == 0) r[(int64_t)rows[i] * NRHS + h] = (int64_t)rr[i][h];
}

// comb[i] = sum_j c_j x_i[j] for every lifted digit vector x_i (the random
// combination whose rational reconstruction gives a divisor of s_n): one
// wave per digit, after the lifting, so the lifting loop carries no extra
// work.  c_j < 2^16, digits < 2^26: the 64-bit sums are exact.
__global__ __launch_bounds__(256) void k_comb_digits(const uint32_t* __restrict__ digits,
                                                     int64_t k, int n,
                                                     const uint32_t* __restrict__ cvec,
                                                     uint64_t* __restrict__ comb) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= k) return;
  const uint32_t* x = digits + i * n;
  uint64_t s = 0;
  for (int j = lane; j < n; j += 64) s += (uint64_t)cvec[j] * x[j];
  s = wave_sum_u64(s);
  if (lane == 0) comb[i] = s;
}

hipError_t launch_comb_digits(const uint32_t* digits, int64_t k, int n, const uint32_t* cvec,
                              uint64_t* comb, hipStream_t st) {
  if (k <= 0 || n <= 0) return hipSuccess;
  k_comb_digits<<<(unsigned)((k + 3) / 4), 256, 0, st>>>(digits, k, n, cvec, comb);
  return hipGetLastError();
}

static bool prime_set(const uint32_t* primes, int np, PrimeSet* ps) {
  if (np < 1 || np > LIFT_MAX_PRIMES || !primes) return false;
  for (int z = 0; z < LIFT_MAX_PRIMES; z++) {
    ps->p[z] = primes[z < np ? z : 0];
    ps->pinv[z] = 1.0 / (double)ps->p[z];
  }
  return true;
}

hipError_t launch_hensel_f64(const int32_t* Ai, const uint32_t* C0, double* E, uint32_t* C1,
                             uint32_t* C2, int n, const uint32_t* primes, int np, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  PrimeSet ps;
  if (!prime_set(primes, np, &ps)) return hipErrorInvalidValue;
  dim3 grid((n + 63) / 64, (n + 63) / 64, np);
  const int64_t nn = (int64_t)n * n;
  k_hensel_f64<0><<<grid, 512, 0, st>>>((const void*)Ai, (const void*)C0, nullptr, n, ps, 0, nn,
                                        0, E);
  k_hensel_f64<1><<<grid, 512, 0, st>>>((const void*)C0, (const void*)E, nullptr, n, ps, nn, nn,
                                        0, C1);
  k_hensel_f64<0><<<grid, 512, 0, st>>>((const void*)Ai, (const void*)C1, E, n, ps, 0, nn, nn, E);
  k_hensel_f64<1><<<grid, 512, 0, st>>>((const void*)C0, (const void*)E, nullptr, n, ps, nn, nn,
                                        0, C2);
  return hipGetLastError();
}

size_t hensel_i8_scratch(int n, int np) {
  const size_t R = (size_t)((n + 63) / 64) * 64;
  return (1 + 4 * (size_t)np) * 3 * R * R;
}

hipError_t launch_hensel_i8(const int32_t* Ai, const uint32_t* C0, double* E, uint32_t* C1,
                            uint32_t* C2, int n, const uint32_t* primes, int np, int8_t* planes,
                            hipStream_t st) {
  if (n <= 0) return hipSuccess;
  PrimeSet ps;
  if (!prime_set(primes, np, &ps) || !planes) return hipErrorInvalidValue;
  for (int z = 0; z < np; z++)
    if (primes[z] > 2u * (uint32_t)LIMB3_MAX + 1u) return hipErrorInvalidValue;
  const int Kp = (n + 63) / 64 * 64;
  const int64_t Rp = Kp, set = 3 * Rp * Kp, nn = (int64_t)n * n;
  if (Kp > 43690) return hipErrorInvalidValue;     // int32 sums: 3 Kp 2^14 < 2^31
  // planes: A (shared), then per prime the sets c0, c0^T, E^T, c1^T
  int8_t* pA = planes;
  int8_t* pc0 = planes + set;
  int8_t* pc0T = pc0 + set;
  int8_t* pET = pc0 + 2 * set;
  int8_t* pc1T = pc0 + 3 * set;
  const int64_t pst = 4 * set;                     // stride between primes
  const dim3 gs(Kp / 64, (unsigned)(Rp / 64), np), gs1(Kp / 64, (unsigned)(Rp / 64), 1);
  const dim3 gm((n + 63) / 64, (n + 63) / 64, np);
  k_split_h<0><<<gs1, 256, 0, st>>>(Ai, 0, n, Kp, Rp, 0, pA, 0, ps);
  k_split_h<1><<<gs, 256, 0, st>>>(C0, nn, n, Kp, Rp, 0, pc0, pst, ps);
  k_split_h<1><<<gs, 256, 0, st>>>(C0, nn, n, Kp, Rp, 1, pc0T, pst, ps);
  k_hensel_i8<0><<<gm, 256, 0, st>>>(pA, pc0T, 0, pst, Rp, Kp, n, ps, nullptr, 0, E);   // E_1
  k_split_h<2><<<gs, 256, 0, st>>>(E, nn, n, Kp, Rp, 1, pET, pst, ps);
  k_hensel_i8<1><<<gm, 256, 0, st>>>(pc0, pET, pst, pst, Rp, Kp, n, ps, nullptr, 0, C1);   // c_1
  k_split_h<1><<<gs, 256, 0, st>>>(C1, nn, n, Kp, Rp, 1, pc1T, pst, ps);
  k_hensel_i8<0><<<gm, 256, 0, st>>>(pA, pc1T, 0, pst, Rp, Kp, n, ps, E, nn, E);          // E_2
  k_split_h<2><<<gs, 256, 0, st>>>(E, nn, n, Kp, Rp, 1, pET, pst, ps);
  k_hensel_i8<1><<<gm, 256, 0, st>>>(pc0, pET, pst, pst, Rp, Kp, n, ps, nullptr, 0, C2);   // c_2
  return hipGetLastError();
}

hipError_t launch_lift_resident3(int grid, const uint32_t* C0, const uint32_t* C1,
                                 const uint32_t* C2, const int32_t* Ai, int64_t* r, uint32_t* rv,
                                 uint32_t* xv, int n, int nrhs, const uint32_t* primes, int np,
                                 int64_t kd, uint32_t* digits, int64_t dig_rhs_stride,
                                 int64_t dig_prime_stride, int* err, hipStream_t st) {
  if (n <= 0 || kd <= 0) return hipSuccess;
  PrimeSet ps;
  if (!prime_set(primes, np, &ps) || nrhs < 1 || nrhs > LIFT3_MAX_RHS) return hipErrorInvalidValue;
  for (int z = 0; z < np; z++)
    if (primes[z] >= (1u << 25)) return hipErrorInvalidValue;
  if (np > 1 && np > lift3_max_primes_of(n)) return hipErrorInvalidValue;
  unsigned spin_limit = 1u << 18;     // polls of about 1 us each: ~0.3 s per wait at most
  int gpp = grid;
  void* args[] = {(void*)&C0, (void*)&C1, (void*)&C2, (void*)&Ai, (void*)&r, (void*)&rv,
                  (void*)&xv, (void*)&n, (void*)&ps, (void*)&gpp, (void*)&kd, (void*)&digits,
                  (void*)&dig_rhs_stride, (void*)&dig_prime_stride, (void*)&err,
                  (void*)&spin_limit};
  const void* f = nullptr;
#define LIFT3_PICK(E)                                                                        \
  f = nrhs == 1 ? (const void*)k_lift_resident3<E, LIFT3_RPW, LIFT3_NWAVE, 1, false>          \
                : (const void*)k_lift_resident3<E, LIFT3_RPW, LIFT3_NWAVE, 2, false>
  if (nrhs > lift3_max_rhs(n)) return hipErrorInvalidValue;
  if (n <= 256) LIFT3_PICK(4);
  else if (n <= 512) LIFT3_PICK(8);
  else if (n <= 1024) LIFT3_PICK(16);
  // above 1024 the third plane and A stay int32 in registers, one
  // right-hand side a launch (the registers of 8 waves a CU hold no more)
  else if (n <= 1536) f = (const void*)k_lift_resident3<24, LIFT3_RPW, LIFT3_NWAVE, 1, true>;
  else if (n <= 2048) f = (const void*)k_lift_resident3<32, LIFT3_RPW, LIFT3_NWAVE, 1, true>;
#undef LIFT3_PICK
  if (!f || grid != lift3_grid_size(n)) return hipErrorInvalidValue;
  return hipLaunchCooperativeKernel(f, dim3(grid * np), dim3(64 * LIFT3_NWAVE), args, 0, st);
}

hipError_t launch_lift_persistent(int grid, const uint32_t* Cu, const int32_t* Ai, int64_t* r,
                                  uint32_t* rp, uint32_t* xbuf, int n, uint32_t p, uint64_t pinv64,
                                  int64_t k, uint32_t* digits, const uint32_t* cvec,
                                  uint64_t* comb, unsigned* bar, int* err, hipStream_t st) {
  if (n <= 0 || k <= 0) return hipSuccess;
  double pinv = 1.0 / (double)p;
  unsigned spin_limit = 1u << 22;     // ~0.1 s of polling per barrier at most
  void* args[] = {(void*)&Cu, (void*)&Ai, (void*)&r, (void*)&rp, (void*)&xbuf, (void*)&n,
                  (void*)&p, (void*)&pinv, (void*)&pinv64, (void*)&k, (void*)&digits,
                  (void*)&cvec, (void*)&comb, (void*)&bar, (void*)&err, (void*)&spin_limit};
  int epl, rpw;
  resident_shape(n, &epl, &rpw);
  const void* f = nullptr;
  if (epl == 4) f = (const void*)k_lift_resident<4, 4>;
  else if (epl == 8) f = (const void*)k_lift_resident<8, 4>;
  else if (epl == 16) f = (const void*)k_lift_resident<16, 2>;
  if (!f || grid != (n + 8 * rpw - 1) / (8 * rpw)) return hipErrorInvalidValue;
  return hipLaunchCooperativeKernel(f, dim3(grid), dim3(512), args, 0, st);
}

}  // namespace detk
