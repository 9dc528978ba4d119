// Shared device code of the LU kernels: lane helpers and the panel
// factorisation body (K2), used by the one-launch-per-step LU
// (lu_kernels.hip) and by the persistent LU over a work queue
// (batch_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <limits.h>
#include <stdint.h>

#include "modp.hpp"

namespace detk {

typedef int v4i_p __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ helpers
// A value that is the same in every lane, moved to scalar registers (an FP64
// VALU operation can take one scalar operand, which saves vector registers).
__device__ __forceinline__ double uniform_d(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The value of one lane (a wave-uniform index) in every lane.
__device__ __forceinline__ double readlane_d(double x, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}

// ------------------------------------------------------------------ K2: panel body
// Factor rows [j0, n) x columns [j0, j0+pb) of every item (m = n - j0 rows).
// One workgroup of T threads per item.  Thread t owns rows t, t+T, ...;
// for each it keeps a window of PB entries of the row in FP64 registers.
// Columns are taken in groups of 8: the group's columns are unrolled (so
// register indices are compile-time constants), and at the end of a group
// the window moves on by 8 columns, which keeps the code small enough for
// the instruction cache.  Finished values (multipliers and pivot rows) go to
// the LDS copy of the panel, sP (int32, m x (PB+1)), written back at the end.
// Pivot = first row at or below the diagonal with a non-zero entry (lowest
// row index); rows are swapped LAPACK-style (whole panel rows).  Row j is
// the pivot unless its entry is 0 mod p, so its owner (thread j) reduces it
// and inverts its entry before the column's barrier; only when row j's entry
// vanishes does a second round fetch the pivot row from below.
// Updates are applied without reduction and every row receives the same
// number of them, each below h^2 (h = (p-1)/2); the window is reduced every
// 8 columns (to |v| <= h + 5 by mod_loose), which keeps every value exact
// (8 h^2 + h + 5 < 2^53 for p < 2^26); the pivot column is reduced before
// use, multipliers and pivot rows fully (|v| <= h).
// Outputs: L below the diagonal, U on and above it, piv[j0+j] = global row
// swapped with row j0+j, the item's flag = 1 if a column has no pivot (det = 0 mod
// p), Linv = the pb x pb unit lower inverse of L11 and, if Uinv != null, the
// upper inverse of U11 (both dense PB x PB, zero-padded).
// The body runs in a workgroup of T threads (T >= 192, a multiple of 64) on
// one item: Wr = the item's slab (row-major, leading dimension ldw), piv_z =
// its pivot record, flag_z = its singularity flag, Linv_z / Uinv_z = its
// PB x PB triangular inverses (Uinv_z may be null), sP = LDS of
// RPT * T * (PB + 1) int32 that holds the finished panel (multipliers and U
// rows, row-major with stride PB + 1) when the body returns.
template <int PB, int RPT, int T>
__device__ __forceinline__ void panel_body(int32_t* __restrict__ Wr, int64_t ldw, int n, int j0,
                                           int pb, double p, double pinv,
                                           int32_t* __restrict__ piv_z,
                                           int32_t* __restrict__ flag_z,
                                           int32_t* __restrict__ Linv_z,
                                           int32_t* __restrict__ Uinv_z, int ncols_sw,
                                           int32_t* __restrict__ sP) {
  constexpr int NW = T / 64;
  constexpr int SP = PB + 1;                  // LDS row stride: odd, so a column is conflict-free
  constexpr int GJ = 8;                       // columns per group (and reduction interval)
  static_assert(PB % GJ == 0 && PB <= 32, "panel width");
  static_assert(T % 64 == 0 && T >= 192, "workgroup size");
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const uint32_t e_inv = (uint32_t)__builtin_amdgcn_readfirstlane((int)((uint32_t)p - 2u));
  int32_t* Wz = Wr + (int64_t)j0 * ldw + j0;
  const int m = n - j0;

  __shared__ double s_prow[2][PB];            // pivot row, reduced (window columns)
  __shared__ double s_old[2][PB];             // row j as it was (moves down when swapped)
  __shared__ double s_inv[2];
  __shared__ int s_min[2][NW];                // each wave's lowest candidate row
  __shared__ double s_dinv[PB];
  __shared__ int s_piv[PB];
  __shared__ int s_sing;
  __shared__ double sBlk[8][PB];              // a group's pivot rows, on their way to lane-per-column
  __shared__ double sU[2][8][PB];             // U rows of a group (window columns), per group parity
  __shared__ double s_gi[2][8];               // pivot inverses of a group
  __shared__ double sRik[8][8];               // a group's pivot-column entries (fraction-free)
  __shared__ int s_gfast[2];

  // each thread loads its own rows straight into registers (16-byte loads of
  // the row's PB entries when the panel is full width: j0, ldw and slab are
  // multiples of 4); the LDS copy of the panel, sP, only ever receives
  // finished values, and every entry of it is written before the write-back
  if (t == 0) s_sing = 0;
  if (t < 2 * PB) s_prow[t / PB][t % PB] = 0.0;   // finite even where it is not written
  if (t < PB) s_dinv[t] = 0.0;
  double a[RPT][PB];
#pragma unroll
  for (int q = 0; q < RPT; q++) {
    const int row = t + q * T;
    const int32_t* src = Wz + (int64_t)(row < m ? row : 0) * ldw;
    // (loads unconditional from the clamped row, the padding selected after:
    // a load under a condition would wait for its own data)
    const bool in = row < m;
    if (pb == PB) {
#pragma unroll
      for (int k4 = 0; k4 < PB / 4; k4++) {
        const v4i_p v = ((const v4i_p*)src)[k4];
        a[q][4 * k4] = in ? (double)v.x : 0.0;
        a[q][4 * k4 + 1] = in ? (double)v.y : 0.0;
        a[q][4 * k4 + 2] = in ? (double)v.z : 0.0;
        a[q][4 * k4 + 3] = in ? (double)v.w : 0.0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < PB; k++) {
        const int32_t v = src[min(k, pb - 1)];
        a[q][k] = (in && k < pb) ? (double)v : 0.0;
      }
    }
  }
  __syncthreads();

  for (int g = 0; g < pb; g += GJ) {
    const int gb = (g / GJ) & 1;
    // ---- The group's pivot rows g..g+7, in wave 0.  Their window entries go
    // through LDS to a lane-per-column layout (lane c: window column c of the
    // eight rows), so that an elimination step needs only the pivot column's
    // entries from other lanes.  A fraction-free elimination of the eight
    // rows (row i <- b_k row_i - r_ik row_k for i > k, b_k and r_ik the pivot
    // column's entries of rows k and i) leaves every row scaled by
    // sigma_k = b_0 ... b_{k-1} at its pivot step, so with one ladder for the
    // eight inverses 1/b_k:
    //   U row k = (row k after step k-1) / sigma_k,  l_ik = r_ik / b_k,
    //   1/a_kk = sigma_k / b_k.
    // This holds while rows g..g+7 are the group's pivots, that is while no
    // b_k is 0 mod p (no swap); gvalid = the number of leading columns for
    // which it holds.  When all eight hold (the fast path) the U rows and the
    // multipliers are stored here, and every other row then takes its eight
    // multipliers and the rank-8 update of its window on its own, after a
    // single barrier.  Values stay |v| <= h + 5 < p through the steps (loose
    // reductions), so v == 0 exactly when p divides v, and products stay
    // below 2^51.
    int gvalid = 0;
    if (wave == 0) {
      if (t >= g && t < g + GJ) {
#pragma unroll
        for (int c = 0; c < PB; c++) sBlk[t - g][c] = a[0][c];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int cl = lane < PB ? lane : PB - 1;
      double F[GJ], bk[GJ];
#pragma unroll
      for (int i = 0; i < GJ; i++) F[i] = sBlk[i][cl];
      int gv = GJ;
#pragma unroll
      for (int k = 0; k < GJ; k++) {
        bk[k] = readlane_d(F[k], k);
        if (bk[k] == 0.0 && gv == GJ) gv = k;
        // the pivot column's entries r_ik (lane k) are kept for the multipliers
        if (lane == k) {
#pragma unroll
          for (int i = k + 1; i < GJ; i++) sRik[i][k] = F[i];
        }
#pragma unroll
        for (int i = k + 1; i < GJ; i++) {
          const double r = readlane_d(F[i], k);
          F[i] = mod_loose(fma(bk[k], F[i], -r * F[k]), p, pinv);
        }
      }
      // 1/b_k in lane k (one ladder for all eight); sigma_k and 1/sigma_k
      double bsel = 1.0;
#pragma unroll
      for (int k = 0; k < GJ; k++) bsel = lane == k ? bk[k] : bsel;
      bsel = bsel == 0.0 ? 1.0 : bsel;                // (columns past gvalid: unused)
      const double ib = pow_mod_fixed(bsel, e_inv, p, pinv);
      double ibk[GJ], sg[GJ], isg[GJ];
#pragma unroll
      for (int k = 0; k < GJ; k++) ibk[k] = readlane_d(ib, k);
      sg[0] = isg[0] = 1.0;
#pragma unroll
      for (int k = 1; k < GJ; k++) {
        sg[k] = mul_mod_loose(sg[k - 1], bk[k - 1], p, pinv);
        isg[k] = mul_mod_loose(isg[k - 1], ibk[k - 1], p, pinv);
      }
      double gi = 0.0;                                // lane k: 1/a_kk
#pragma unroll
      for (int k = 0; k < GJ; k++) gi = lane == k ? mul_mod(sg[k], ibk[k], p, pinv) : gi;
      if (lane < GJ) s_gi[gb][lane] = gi;
      gvalid = gv;
      const bool fastg = gv == GJ && g + GJ <= pb;
      if (fastg) {
#pragma unroll
        for (int k = 0; k < GJ; k++) {
          const double u = mul_mod(F[k], isg[k], p, pinv);             // U row g+k (lanes >= k)
          if (lane < PB) sU[gb][k][lane] = u;
          if (lane >= k && lane < PB && g + lane < pb) sP[(g + k) * SP + g + lane] = (int32_t)u;
        }
        // multipliers of the block: lane i*8+k stores l_ik = r_ik / b_k (i > k)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        {
          const int i = lane / GJ, k = lane % GJ;
          const double ibl = __shfl(ib, k);
          if (i > k) sP[(g + i) * SP + g + k] = (int32_t)mul_mod(sRik[i][k], ibl, p, pinv);
        }
        if (lane < GJ) {
          s_piv[g + lane] = g + lane;
          s_dinv[g + lane] = gi;
        }
      }
      if (lane == 0) s_gfast[gb] = fastg ? 1 : 0;
    }
    __syncthreads();
    if (s_gfast[gb]) {
      // every row: multipliers l_k = (a_k - sum_{m<k} l_m U_mk) / U_kk, then
      // a_c -= sum_k l_k U_kc for the window columns past the group (eight
      // pending products, below 2^51, reduced at the window shift); rows at
      // or above g+7 and absent rows run through and store nothing
      double inv[GJ];
#pragma unroll
      for (int k = 0; k < GJ; k++) inv[k] = s_gi[gb][k];
      double l[RPT][GJ];
#pragma unroll
      for (int k = 0; k < GJ; k++) {
#pragma unroll
        for (int q = 0; q < RPT; q++) {
          double v = a[q][k];
#pragma unroll
          for (int mm = 0; mm < k; mm++) v = fma(-l[q][mm], sU[gb][mm][k], v);
          l[q][k] = mul_mod_loose(mod_loose(v, p, pinv), inv[k], p, pinv);   // |l| <= h + 5
        }
      }
      // canonical multipliers for the store and the update (eight products
      // of |l| <= h stay below 2^53 for p < 2^26)
#pragma unroll
      for (int k = 0; k < GJ; k++)
#pragma unroll
        for (int q = 0; q < RPT; q++) l[q][k] = mod_c(l[q][k], p, pinv);
#pragma unroll
      for (int q = 0; q < RPT; q++) {
        const int row = t + q * T;
        if (row >= g + GJ && row < m) {
#pragma unroll
          for (int k = 0; k < GJ; k++) sP[row * SP + g + k] = (int32_t)l[q][k];
        }
      }
#pragma unroll
      for (int c = GJ; c < PB; c++) {
#pragma unroll
        for (int k = 0; k < GJ; k++) {
          const double u = sU[gb][k][c];
#pragma unroll
          for (int q = 0; q < RPT; q++) a[q][c] = fma(-l[q][k], u, a[q][c]);
        }
      }
    } else {
#pragma unroll
    for (int jj = 0; jj < GJ; jj++) {
      const int j = g + jj;
      if (j < pb) {
        const int buf = jj & 1;
        // lowest row of this wave at or below j with a non-zero entry (the
        // reduction runs on every row: finished rows are never read again)
        int wc = INT_MAX;
#pragma unroll
        for (int q = RPT - 1; q >= 0; q--) {
          const int row = t + q * T;
          a[q][jj] = mod_loose(a[q][jj], p, pinv);    // exact zero test (|r| < p)
          const uint64_t bal = __ballot(row >= j && row < m && a[q][jj] != 0.0);
          if (bal) wc = q * T + wave * 64 + (__ffsll((unsigned long long)bal) - 1);
        }
        // row j (thread j, since j < PB <= 64): publish it as it is; if its
        // entry is non-zero it is the pivot, so reduce it and invert the entry
        if (wave == 0) {
          if (t == j) {
#pragma unroll
            for (int k = 0; k < PB; k++)
              if (k >= jj) s_old[buf][k] = a[0][k];
            if (wc == j) s_inv[buf] = jj < gvalid ? s_gi[gb][jj] : pow_mod_fixed(a[0][jj], e_inv, p, pinv);
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
          if (wc == j && lane >= jj && lane < PB)
            s_prow[buf][lane] = mod_c(s_old[buf][lane], p, pinv);
        }
        if (lane == 0) s_min[buf][wave] = wc;
        __syncthreads();
        int pr = INT_MAX;
#pragma unroll
        for (int w = 0; w < NW; w++) pr = min(pr, s_min[buf][w]);
        pr = __builtin_amdgcn_readfirstlane(pr);      // the same in every lane
        const bool singular = pr == INT_MAX;          // no pivot: det = 0 mod p, row j kept
        if (singular) pr = j;
        if (pr != j || singular) gvalid = 0;          // the group's later pivots change
        if (pr != j) {                                // pivot below row j: second round
          if (wave == ((pr % T) >> 6)) {
            const int qp = pr / T;
#pragma unroll
            for (int q = 0; q < RPT; q++)
              if (q == qp && t + q * T == pr) {
#pragma unroll
                for (int k = 0; k < PB; k++)
                  if (k >= jj) s_prow[buf][k] = a[q][k];
                s_inv[buf] = inv_mod_call(a[q][jj], e_inv, p, pinv);
              }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (lane > jj && lane < PB) s_prow[buf][lane] = mod_c(s_prow[buf][lane], p, pinv);
            // old row j moves down to row pr (its entry j is 0 mod p)
#pragma unroll
            for (int q = 0; q < RPT; q++)
              if (q == qp && t + q * T == pr) {
                a[q][jj] = 0.0;
#pragma unroll
                for (int k = 1; k < PB; k++)
                  if (k > jj) a[q][k] = s_old[buf][k];
              }
          }
          __syncthreads();
          // swap the finished (multiplier) parts of rows j and pr
          if (t < j) {
            const int32_t v = sP[j * SP + t];
            sP[j * SP + t] = sP[pr * SP + t];
            sP[pr * SP + t] = v;
          }
        }
        // with no pivot, row j stays (U row j = row j) and nothing is eliminated
        const double inv = uniform_d(singular ? 0.0 : s_inv[buf]);
        if (t < pb - j)                                                            // U row j
          sP[j * SP + j + t] = (int32_t)mod_c(singular ? s_old[buf][jj + t] : s_prow[buf][jj + t], p, pinv);
        double pv[PB];                                // pivot row (same in all lanes)
#pragma unroll
        for (int k = 1; k < PB; k++)
          if (k > jj) pv[k] = s_prow[buf][k];   // any finite values when singular
        // elimination on every row (rows at or above j, and absent rows, are
        // never read again); only the multipliers of live rows are stored
#pragma unroll
        for (int q = 0; q < RPT; q++) {
          const int row = t + q * T;
          const double l = mul_mod(a[q][jj], inv, p, pinv);
          if (row > j && row < m) sP[row * SP + j] = (int32_t)l;
#pragma unroll
          for (int k = 1; k < PB; k++)
            if (k > jj) a[q][k] = fma(-l, pv[k], a[q][k]);
        }
        if (t == 0) {                   // results stay in LDS until the end (no global
          s_dinv[j] = inv;              // stores inside the loop)
          s_piv[j] = pr;
          if (singular) s_sing = 1;
        }
      }
    }
    }
    // next window: columns g+8 .. g+8+PB-1, reduced (at most 8 updates pending)
#pragma unroll
    for (int q = 0; q < RPT; q++)
#pragma unroll
      for (int k = 0; k < PB; k++)
        a[q][k] = (k + GJ < PB) ? mod_loose(a[q][k + GJ], p, pinv) : 0.0;
  }
  __syncthreads();
  // Waves 2.. write the panel back (four consecutive columns a thread, 16-byte
  // stores: j0, ldw and slab are multiples of 4) while waves 0 and 1 compute
  // the triangular inverses below.
  if (wave >= 2) {
    constexpr int PB4 = PB / 4;
    for (int e = t - 128; e < m * PB4; e += T - 128) {
      const int r = e / PB4, k = (e % PB4) * 4;
      int32_t* dst = Wz + (int64_t)r * ldw + k;
      const int32_t* src = sP + r * SP + k;
      if (k + 3 < pb) {
        *(v4i_p*)dst = v4i_p{src[0], src[1], src[2], src[3]};
      } else {
#pragma unroll
        for (int u = 0; u < 4; u++)
          if (k + u < pb) dst[u] = src[u];
      }
    }
  }
  if (t < pb) piv_z[j0 + t] = j0 + s_piv[t];
  if (t == 0 && s_sing) *flag_z = 1;
  // Triangular inverses, lane c of wave 0 (Linv) or wave 1 (Uinv) solving
  // for one column with the column in registers.  Wave 0 solves L X = I;
  // wave 1 solves U^T Y = I (U^T is lower triangular with the pivots on its
  // diagonal), whose column c is row c of U^{-1}:
  //   x = e_c; for k = 0..pb-1: x[k] = x[k] / diag[k] (final);
  //            x[i] -= M[i][k] x[k] for i > k
  // Entries are reduced every 8 steps (8 h^2 + h + 5 < 2^53).
  if (wave < 2 && lane < PB && (wave == 0 || Uinv_z != nullptr)) {
    const bool up = wave == 1;
    const int cc = lane;
    double x[PB];
#pragma unroll
    for (int i = 0; i < PB; i++) x[i] = (i == cc) ? 1.0 : 0.0;
    // no masks needed: for L, rows i >= pb never feed rows below pb (and are
    // not written out); for U^T, columns >= pb of sP are 0 and so is dinv
    if (!up) {
#pragma unroll
      for (int k = 0; k < PB; k++) {
        x[k] = mod_c(x[k], p, pinv);
#pragma unroll
        for (int i = 1; i < PB; i++)
          if (i > k) x[i] = fma(-(double)sP[i * SP + k], x[k], x[i]);
        if ((k & 7) == 7) {
#pragma unroll
          for (int i = 1; i < PB; i++)
            if (i > k) x[i] = mod_loose(x[i], p, pinv);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < PB; k++) {
        x[k] = mul_mod(mod_c(x[k], p, pinv), s_dinv[k], p, pinv);
#pragma unroll
        for (int i = 1; i < PB; i++)
          if (i > k) x[i] = fma(-(double)sP[k * SP + i], x[k], x[i]);
        if ((k & 7) == 7) {
#pragma unroll
          for (int i = 1; i < PB; i++)
            if (i > k) x[i] = mod_loose(x[i], p, pinv);
        }
      }
    }
    int32_t* out = up ? Uinv_z : Linv_z;
#pragma unroll
    for (int i = 0; i < PB; i++)
      out[up ? cc * PB + i : i * PB + cc] = (i < pb && cc < pb) ? (int32_t)x[i] : 0;
  }
  // The panel's row swaps on the columns [j0 + pb, ncols_sw) right of it,
  // when the caller asks for them (ncols_sw > 0) and a pivot came from below
  // (random inputs almost never need it): one column a thread, the swaps in
  // order.
  if (ncols_sw > j0 + pb) {
    __syncthreads();
    bool any = false;
    for (int i = 0; i < pb; i++) any |= s_piv[i] != i;
    if (any) {
      for (int c = j0 + pb + t; c < ncols_sw; c += T)
        for (int i = 0; i < pb; i++) {
          const int r = s_piv[i];
          if (r != i) {
            int32_t* a0 = Wr + (int64_t)(j0 + i) * ldw + c;
            int32_t* a1 = Wr + (int64_t)(j0 + r) * ldw + c;
            const int32_t v = *a0;
            *a0 = *a1;
            *a1 = v;
          }
        }
    }
  }
}

// ------------------------------------------------------------------ diagonal block body
// Factors the pb x pb diagonal block (pb <= 32) whose top-left entry is Wb
// (leading dimension ldw) without a pivot search below it.  Two eliminations
// run side by side, each held whole by one wave, so a step needs no exchange
// between waves and no barrier: [A11 | I] in wave 0 and [A11^T | I] in wave 1
// (a block narrower than 32 is padded with the identity).  A fraction-free
// elimination, row_i <- b_k row_i - r_ik row_k for i > k with b_k = the
// pivot-column entry of row k, leaves row i scaled by sigma_i = b_0 ...
// b_{i-1}, so no inverse is needed inside the loop:
//  - [A11 | I] gives [U | L^{-1}] row by row after the scaling 1 / sigma_i;
//  - A11^T = L_T U_T with L_T = U'^T and U_T = D L^T (U = D U', D =
//    diag(u_ii), U' unit upper), whose pivots, and so whose b_i, are those of
//    A11; [A11^T | I] gives L_T^{-1} = (U'^{-1})^T after the scaling
//    1 / sigma_i, and U^{-1} = U'^{-1} D^{-1} with u_ii = b_i / sigma_i, so
//    U^{-1}[c][i] = (row i of the second elimination)[c] / b_i.
// Layout.  At step k the live columns of [A11 | I] are the left columns
// k..31 and the right columns 32..32+k: the left column k is eliminated at
// step k (its entries below row k become 0), and the right column 32+k is
// zero outside row k (where it holds sigma_k) until step k.  So one lane
// holds the left column c until step c and the right column 32+c from then
// on, and 32 lanes hold the whole block: at step c lane c updates its rows
// below c as b' = 0, pivot-row entry sigma_c, which turns them into the
// right column's -r_ic sigma_c.  Rows above c keep U's column c, and row c
// keeps b_c (U's diagonal) in wave 0 or sigma_c (the right column's entry,
// wanted for U^{-1}[c][c]) in wave 1.  The two 32-lane halves of a wave then
// split the rows: lanes 0..31 hold rows 0..15 and lanes 32..63 rows 16..31
// (lane = column c & 31, slot s = row s + 16 * half), and one instruction
// updates a row of each half.  The multipliers r_ik come from lane k of the
// same half by ds_swizzle (issued right after the row's previous update, so
// they are in flight during the rest of the step), the pivot row of the
// upper half reaches the lower half by ds_bpermute.  While k < 16 the upper
// half also runs the updates of its finished rows (its slots <= k); their
// results are discarded (each upper row is copied out when it becomes final,
// at the start of its own step), which keeps every step one instruction
// stream with no lane masking.  Steps 16 and later issue only the slots of
// rows still below the pivot.
// The 32 inverses a wave needs (1 / sigma_i in wave 0, 1 / b_i in wave 1)
// come from one Fermat ladder run by the lanes side by side (lane c of half
// h for index (c + 16 h) mod 32, so that the scale of slot s is read from lane
// s of either half); sigma_i is the running product of the pivots, kept beside
// the elimination.
// Outputs: U11 into the block (on and above the diagonal), L11^{-1} at Lz
// (32 x 32 row-major, only its entries below the diagonal: it is unit lower
// triangular, and its reader takes the rest as given), U11^{-1} dense 32 x 32
// row-major at Uz (zero outside pb x pb),
// piv_z[j0 + i] = j0 + i, *flag = 1 when a pivot is 0 mod p (the caller then
// runs the full pivot search).  Values stay below (p + 9) / 2 in magnitude
// through the loose reductions, so every product is below 2^52.  Waves 2 and
// up of the workgroup do nothing here; no LDS memory is used (the swizzles
// and permutes only use its crossbar).

// x from lane K of each 32-lane half (ds_swizzle, bitmask mode: and 0, or K).
template <int K>
__device__ __forceinline__ double bcast_half(double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)u, K << 5);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_swizzle((int)(uint32_t)(u >> 32), K << 5);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// x from the lane whose byte address is addr (ds_bpermute).
__device__ __forceinline__ double bpermute_d(int addr, double x) {
  const uint64_t u = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// State of the elimination carried from step to step.
struct DiagElim {
  double X[16];      // slot s: row s + 16 * half of this lane's column
  double M[16];      // the next step's multipliers (its pivot column, per slot)
  double F[16];      // upper half: row s as it was when it became final
  double xkn;        // lower half: the next pivot row's entry, from the upper half
  double bnext;      // the next pivot b_k (uniform)
  double S;          // running product of the pivots (uniform)
  double sig, bl;    // sigma_j and b_j for this lane's ladder index j
  bool zero;
};

// Step K, then the steps after it (a compile-time recursion, so that every
// slot index is a register).  Within a step the slots go in groups of G,
// each phase over the group before the next, so that independent FP64 chains
// fill the pipeline; a scheduling barrier between steps and between groups
// keeps the compiler from chaining one slot through several steps (which
// would wait on every swizzle).
template <int K, int G>
__device__ __forceinline__ void diag_elim_step(DiagElim& e, int L, int h, int xaddr, bool tr,
                                               double p, double pinv) {
  if constexpr (K < 32) {
    constexpr double RND = 6755399441055744.0;
    constexpr int hK = K >> 4, sK = K & 15;
    constexpr int K1 = K + 1, hK1 = K1 >> 4, sK1 = K1 & 15;
    __builtin_amdgcn_sched_barrier(0);
    const double braw = e.bnext;
    e.zero |= braw == 0.0;
    const double bk = braw == 0.0 ? 1.0 : braw;      // (the result is discarded then)
    const bool atK = L == K;
    const double Sk = e.S;                           // sigma_K
    double xk;                                       // pivot row K, this lane's column
    if constexpr (hK == 0) {
      const double own = e.X[sK];
      xk = h ? e.xkn : own;
      e.F[sK] = (atK && tr) ? Sk : own;
    } else {
      xk = e.X[sK];
    }
    const bool jK = ((L + 16 * h) & 31) == K;
    e.sig = jK ? Sk : e.sig;
    e.bl = jK ? bk : e.bl;
    const double bkp = atK ? 0.0 : bk;
    const double xkp = atK ? Sk : xk;
    e.S = mul_mod_loose(e.S, bk, p, pinv);
    constexpr int s0 = hK == 0 ? 0 : sK + 1;
#pragma unroll
    for (int i0 = s0; i0 < 16; i0 += G) {
      double x[G], q[G];
#pragma unroll
      for (int j = 0; j < G; j++)
        if (i0 + j < 16) x[j] = -e.M[i0 + j] * xkp;
#pragma unroll
      for (int j = 0; j < G; j++)
        if (i0 + j < 16) x[j] = fma(bkp, e.X[i0 + j], x[j]);
#pragma unroll
      for (int j = 0; j < G; j++)
        if (i0 + j < 16) q[j] = fma(x[j], pinv, RND);
#pragma unroll
      for (int j = 0; j < G; j++)
        if (i0 + j < 16) q[j] = q[j] - RND;
#pragma unroll
      for (int j = 0; j < G; j++)
        if (i0 + j < 16) {
          e.X[i0 + j] = fma(-q[j], p, x[j]);
          if constexpr (K1 < 32) {
            e.M[i0 + j] = bcast_half<K1>(e.X[i0 + j]);
            if (i0 + j == sK1) {
              e.bnext = readlane_d(e.X[i0 + j], hK1 * 32 + K1);
              if constexpr (K1 < 16) e.xkn = bpermute_d(xaddr, e.X[i0 + j]);
            }
          }
        }
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (hK == 1) e.X[sK] = (atK && tr) ? Sk : e.X[sK];
    diag_elim_step<K + 1, G>(e, L, h, xaddr, tr, p, pinv);
  }
}

// a^e mod p by the right-to-left ladder over the nb low bits of e (nb uniform).
__device__ __forceinline__ double pow_mod_nbits(double a, uint32_t e, int nb, double p,
                                                double pinv) {
  double r = 1.0, b = a;
  for (int i = 0; i < nb; i++) {
    const double rb = mul_mod_loose(r, b, p, pinv);
    r = ((e >> i) & 1u) ? rb : r;
    b = mul_mod_loose(b, b, p, pinv);
  }
  return mod_c(r, p, pinv);
}

// x from lane s of each 32-lane half, s = 0..15.
__device__ __forceinline__ void bcast_half16(double x, double (&out)[16]) {
  out[0] = bcast_half<0>(x);   out[1] = bcast_half<1>(x);   out[2] = bcast_half<2>(x);
  out[3] = bcast_half<3>(x);   out[4] = bcast_half<4>(x);   out[5] = bcast_half<5>(x);
  out[6] = bcast_half<6>(x);   out[7] = bcast_half<7>(x);   out[8] = bcast_half<8>(x);
  out[9] = bcast_half<9>(x);   out[10] = bcast_half<10>(x); out[11] = bcast_half<11>(x);
  out[12] = bcast_half<12>(x); out[13] = bcast_half<13>(x); out[14] = bcast_half<14>(x);
  out[15] = bcast_half<15>(x);
}

__device__ __forceinline__ void diag_block_body(int32_t* __restrict__ Wb, int64_t ldw, int pb,
                                                double p, double pinv, int32_t* __restrict__ piv_z,
                                                int j0, int32_t* __restrict__ flag,
                                                int32_t* __restrict__ Lz, int32_t* __restrict__ Uz) {
  const int t = threadIdx.x;
  const int c = t & 63, w = t >> 6;
  if (w >= 2) return;
  const bool tr = w == 1;                            // the transposed elimination
  const int L = c & 31, h = c >> 5;
  const int ld = (int)ldw;                           // (the block lies in the first 2^31 entries)
  const uint32_t e_inv = (uint32_t)__builtin_amdgcn_readfirstlane((int)((uint32_t)p - 2u));
  const int nb = 32 - __builtin_clz(e_inv | 1u);
  DiagElim e;
  {
    // every load is issued before any is used (clamped indices stay inside
    // the pb x pb block; the padding is selected afterwards)
    int32_t v[16];
    const int cc = min(L, pb - 1);
#pragma unroll
    for (int s = 0; s < 16; s++) {
      const int ii = min(s + 16 * h, pb - 1);
      v[s] = Wb[tr ? cc * ld + ii : ii * ld + cc];
    }
#pragma unroll
    for (int s = 0; s < 16; s++) {
      const int r = s + 16 * h;
      e.X[s] = (r < pb && L < pb) ? (double)v[s] : (L == r ? 1.0 : 0.0);
    }
  }
  const int xaddr = (c ^ 32) << 2;
#pragma unroll
  for (int s = 0; s < 16; s++) e.M[s] = bcast_half<0>(e.X[s]);
  e.xkn = bpermute_d(xaddr, e.X[0]);
  e.bnext = readlane_d(e.X[0], 0);
  e.S = 1.0;
  e.sig = 1.0;
  e.bl = 1.0;
  e.zero = false;
  diag_elim_step<0, 8>(e, L, h, xaddr, tr, p, pinv);
  // lane c of half h: 1 / sigma_j (wave 0) or 1 / b_j (wave 1), j = (c + 16 h) mod 32
  const double y = pow_mod_nbits(tr ? e.bl : e.sig, e_inv, nb, p, pinv);
  double ys[16];
  bcast_half16(y, ys);
  double R[16];
#pragma unroll
  for (int s = 0; s < 16; s++) R[s] = mul_mod(h ? e.X[s] : e.F[s], ys[s], p, pinv);
  const bool lin = L < pb;
  if (!tr) {
    // row r: U[r][L] for L >= r (into the block), L^{-1}[r][L] for L < r,
    // one store a row (each lane writes one of the two)
#pragma unroll
    for (int s = 0; s < 16; s++) {
      const int r = s + 16 * h;
      const int32_t v = (int32_t)R[s];
      const bool up = L >= r;
      int32_t* const dst = up ? Wb + r * ld + L : Lz + r * 32 + L;
      if (!up || lin) *dst = v;
    }
  } else {
    // U^{-1}[L][r] for r >= L
#pragma unroll
    for (int s = 0; s < 16; s++) {
      const int r = s + 16 * h;
      Uz[L * 32 + r] = (r >= L && r < pb && lin) ? (int32_t)R[s] : 0;
    }
  }
  if (t < pb) piv_z[j0 + t] = j0 + t;
  if (e.zero && t == 0) *flag = 1;
}

}  // namespace detk
