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
