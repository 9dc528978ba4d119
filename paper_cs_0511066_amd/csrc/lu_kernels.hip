// Blocked LU modulo p over a batch of primes, for gfx950.
//
// Section 2.1 of the paper obtains each modular determinant det(A) mod p_i
// from an LU factorisation modulo p_i; Section 6 notes that the LU runs of
// one CRA step are independent.  Here one batch item is one (matrix, prime)
// pair, and every kernel covers all items of a batch in one launch.
//
// Storage: item z owns a slab W + z*slab of `rows` x ldw int32 centred
// residues, row-major.  Two-level right-looking blocking:
//   outer block of width NB  : tri_inv (L11^{-1}), trsm_apply (U12), gemm (A22)
//   inner panel of width PB  : panel (pivot/scale/rank-1 in registers),
//                              swaps, trsm_apply and gemm inside the block.
// The trailing update A22 -= L21 U12 is the dense contraction: FP64 MFMA
// (16x16x4) with the sum of |products| kept <= 2^53 per reduction chunk, or
// int8 MFMA (16x16x64) on three signed limbs with int32 accumulation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>
#include <limits.h>

#include "modp.hpp"
#include "kernels.hpp"
#include "panel.hpp"
#include "i8tile.hpp"

namespace detk {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef int v4i __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ K1: residues
// W[z][i][j] = A[i][j] mod p_z (centred) for j < n; columns n <= j < ncols
// hold the identity's columns j - n (the right half of [A | I] for ncols =
// 2n; zero from column 2n on).
__global__ void k_residues(const int64_t* __restrict__ A, int64_t lda, int n, int ncols,
                           int32_t* __restrict__ W, int64_t ldw, int64_t slab,
                           const Modulus* __restrict__ mods, int nitems) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= ncols || i >= n) return;
  double a;
  if (j < n) a = (double)A[(int64_t)i * lda + j];   // |a| < 2^31: exact
  else a = (j - n == i) ? 1.0 : 0.0;
  for (int z = 0; z < nitems; z++) {
    const double p = mods[z].p, pinv = mods[z].pinv;
    W[(int64_t)z * slab + (int64_t)i * ldw + j] = (int32_t)mod_c(a, p, pinv);
  }
}

// ------------------------------------------------------------------ K2: panel
// One 512-thread workgroup per batch item runs the panel body (panel.hpp).
template <int PB, int RPT>
__global__ __launch_bounds__(512) void k_panel(int32_t* __restrict__ W, int64_t ldw, int64_t slab,
                                                int n, int j0, int pb,
                                                const Modulus* __restrict__ mods,
                                                int32_t* __restrict__ piv, int64_t piv_stride,
                                                int32_t* __restrict__ flags,
                                                int32_t* __restrict__ Linv,
                                                int32_t* __restrict__ Uinv, int ncols_sw) {
  __shared__ int32_t sP[RPT * 512 * (PB + 1)];
  const int z = blockIdx.x;
  panel_body<PB, RPT, 512>(W + (int64_t)z * slab, ldw, n, j0, pb, mods[z].p, mods[z].pinv,
                           piv + (int64_t)z * piv_stride, flags + z, Linv + (int64_t)z * PB * PB,
                           Uinv ? Uinv + (int64_t)z * PB * PB : nullptr, ncols_sw, sP);
}

// ------------------------------------------------------------------ K2': diagonal block
// One two-wave workgroup per item factors the pb x pb diagonal block at
// (j0, j0) without a pivot search below it (diag_block_body, panel.hpp), for
// an LU whose update forms L21 itself (k_lu_update with Uinv).
__global__ __launch_bounds__(128) void k_diag_block(int32_t* __restrict__ W, int64_t ldw,
                                                    int64_t slab, int j0, int pb,
                                                    const Modulus* __restrict__ mods,
                                                    int32_t* __restrict__ piv, int64_t piv_stride,
                                                    int32_t* __restrict__ flags,
                                                    int32_t* __restrict__ Linv,
                                                    int32_t* __restrict__ Uinv) {
  const int z = blockIdx.x;
  diag_block_body(W + (int64_t)z * slab + (int64_t)j0 * ldw + j0, ldw, pb, mods[z].p,
                  mods[z].pinv, piv + (int64_t)z * piv_stride, j0, flags + z,
                  Linv + (int64_t)z * 1024, Uinv + (int64_t)z * 1024);
}

// ------------------------------------------------------------------ K3: row swaps
// Apply the swaps of panel [j0, j0+pb) (row j0+j <-> piv[j0+j], in order) to
// the columns [c0a, c1a) and [c0b, c1b) of every item.
__global__ void k_swaps(int32_t* __restrict__ W, int64_t ldw, int64_t slab, int j0, int pb,
                        const int32_t* __restrict__ piv, int64_t piv_stride,
                        int c0a, int c1a, int c0b, int c1b) {
  const int z = blockIdx.y;
  const int32_t* pz = piv + (int64_t)z * piv_stride + j0;
  // one pivot a thread (pb <= 32 <= blockDim.x)
  const int tt = threadIdx.x;
  if (!__syncthreads_or(tt < pb && pz[tt] != j0 + tt)) return;
  const int wa = c1a - c0a;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int wtot = wa + (c1b - c0b);
  if (idx >= wtot) return;
  const int col = idx < wa ? c0a + idx : c0b + (idx - wa);
  int32_t* Wz = W + (int64_t)z * slab + col;
  for (int j = 0; j < pb; j++) {
    const int r = pz[j];
    if (r != j0 + j) {
      const int32_t v = Wz[(int64_t)(j0 + j) * ldw];
      Wz[(int64_t)(j0 + j) * ldw] = Wz[(int64_t)r * ldw];
      Wz[(int64_t)r * ldw] = v;
    }
  }
}

// ------------------------------------------------------------------ triangular inverse
// Inverse of the unit lower kb x kb block L11 at rows/cols [k0, k0+kb) of
// every item (kb <= 128).  One workgroup per item; wave w computes columns
// w, w+16, ...  For column c the forward substitution
//   X[c][c] = 1,  X[i][c] = -sum_{k=c}^{i-1} L[i][k] X[k][c]
// is sequential in i; each sum is split over the 64 lanes (lane l takes
// k = c+l and c+l+64), reduced per lane and then across the wave, so every
// partial sum stays far below 2^53.  Lane l keeps X[l][c] and X[l+64][c].
// Out: Tinv[z] dense ldt x ldt (zero outside kb x kb).
__global__ __launch_bounds__(1024) void k_tri_inv(const int32_t* __restrict__ W, int64_t ldw,
                                                  int64_t slab, int k0, int kb,
                                                  const Modulus* __restrict__ mods,
                                                  int32_t* __restrict__ Tinv, int ldt) {
  const int z = blockIdx.x;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const double p = mods[z].p, pinv = mods[z].pinv;
  __shared__ double sT[128][129];
  const int32_t* Wz = W + (int64_t)z * slab + (int64_t)k0 * ldw + k0;
  for (int e = t; e < 128 * 128; e += 1024) {
    const int i = e >> 7, k = e & 127;
    sT[i][k] = (i < kb && k < i) ? (double)Wz[(int64_t)i * ldw + k] : 0.0;
  }
  __syncthreads();
  int32_t* Tz = Tinv + (int64_t)z * ldt * ldt;
  for (int c = wave; c < ldt; c += 16) {
    double x0 = (lane == c) ? 1.0 : 0.0;             // X[lane][c]
    double x1 = (lane + 64 == c) ? 1.0 : 0.0;        // X[lane + 64][c]
    if (c < kb) {
      for (int i = c + 1; i < kb; i++) {
        // X[k][c] lives in lane k mod 64 (x0 for k < 64, x1 for k >= 64)
        const int k1 = c + lane, k2 = k1 + 64;
        const int src = k1 & 63;
        const double v0 = __shfl(x0, src, 64), v1 = __shfl(x1, src, 64);
        const double t1 = sT[i][min(k1, 127)], t2 = sT[i][min(k2, 127)];
        double s = (k1 < i) ? t1 * (k1 < 64 ? v0 : v1) : 0.0;
        s = (k2 < i) ? fma(t2, v1, s) : s;
        s = mod_c(s, p, pinv);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        const double xi = mod_c(-s, p, pinv);
        if (i < 64) {
          if (lane == i) x0 = xi;
        } else if (lane == i - 64) {
          x1 = xi;
        }
      }
    }
    if (lane < ldt) Tz[lane * ldt + c] = (c < kb && lane < kb) ? (int32_t)x0 : 0;
    if (lane + 64 < ldt) Tz[(lane + 64) * ldt + c] = (c < kb && lane + 64 < kb) ? (int32_t)x1 : 0;
  }
}

// ------------------------------------------------------------------ FP64 MFMA tile machinery
// A workgroup computes a 64x64 tile, each wave a rectangle of MFMA 16x16
// blocks.  Operands are staged in LDS as doubles, k-major, so that a lane
// reads 16 consecutive doubles per row.
// v_mfma_f64_16x16x4: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// result element r of lane l is D[l/16 + 4r][l%16].
constexpr int GB_M = 64, GB_N = 64, GB_K = 32;

// ------------------------------------------------------------------ general modular product
// C <op> A B (mod p) on int32 centred residues of one slab per item, FP64
// MFMA on 64x64 tiles, K in chunks of 32 with the next chunk's global loads
// issued before the current chunk's MFMAs (latency hidden for long K).
// Sums are reduced every kc4 MFMA k-steps (sums of |products| stay <= 2^53).
// op: 0 C -= AB, 1 C += AB, 2 C = AB, 3 C = -AB.  upper_a: A is upper
// triangular (zero below the diagonal), so a row tile starts K at its row.
// Items: z = blockIdx.z = zo nin + zi at W + zo slab_out + zi slab, with
// modulus mods[zo] (mod_by_outer) or mods[z].
constexpr int GM_K = 32;
// WR x WC waves, each an MI x NJ grid of 16 x 16 MFMA blocks: tiles of
// 16 MI WR x 16 NJ WC (64 x 64 with four waves of 2 x 2 blocks, or with
// eight waves of 2 x 1 blocks, two waves a SIMD).
template <int WR, int WC, int MI, int NJ>
__global__ __launch_bounds__(64 * WR * WC) void k_gemm_mod(int32_t* __restrict__ W, int64_t slab,
                                                           int64_t offC, int64_t offA,
                                                           int64_t offB, int64_t ldw, int M,
                                                           int N, int K,
                                                           const Modulus* __restrict__ mods,
                                                           int kc4, int op, int upper_a, int nin,
                                                           int64_t slab_out, int mod_by_outer) {
  constexpr int T = 64 * WR * WC, TM = 16 * MI * WR, TN = 16 * NJ * WC;
  constexpr int NL = TM * GM_K / T, NR = GM_K * TN / T;
  const int z = blockIdx.z;
  const int zo = z / nin, zi = z - zo * nin;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const Modulus& md = mods[mod_by_outer ? zo : z];
  const double p = md.p, pinv = md.pinv;
  int32_t* Wz = W + (int64_t)zo * slab_out + (int64_t)zi * slab;
  const int32_t* Ag = Wz + offA;
  const int32_t* Bg = Wz + offB;
  int32_t* Cg = Wz + offC;
  const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
  __shared__ double sA[GM_K][TM + 2];
  __shared__ double sB[GM_K][TN + 2];
  int32_t areg[NL], breg[NR];
  // value u of thread t: element u * T + t of the tile, row-major.  The
  // loads are unconditional from indices clamped into range (M, N, K >= 1;
  // a load under a condition would wait for its data at once) and the
  // padding is applied when the values are stored to LDS.
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int f = u * T + t, r = f / GM_K, k = f % GM_K;
      areg[u] = Ag[(int64_t)min(row0 + r, M - 1) * ldw + min(k0 + k, K - 1)];
    }
#pragma unroll
    for (int u = 0; u < NR; u++) {
      const int f = u * T + t, k = f / TN, c = f % TN;
      breg[u] = Bg[(int64_t)min(k0 + k, K - 1) * ldw + min(col0 + c, N - 1)];
    }
  };
  v4d acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; i++)
#pragma unroll
    for (int j = 0; j < NJ; j++) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
  const int kbeg = upper_a ? (row0 / GM_K) * GM_K : 0;
  int steps = 0;
  if (kbeg < K) gload(kbeg);
  for (int k0 = kbeg; k0 < K; k0 += GM_K) {
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int f = u * T + t, r = f / GM_K, k = f % GM_K;
      sA[k][r] = (row0 + r < M && k0 + k < K) ? (double)areg[u] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NR; u++) {
      const int f = u * T + t, k = f / TN, c = f % TN;
      sB[k][c] = (k0 + k < K && col0 + c < N) ? (double)breg[u] : 0.0;
    }
    __syncthreads();
    if (k0 + GM_K < K) gload(k0 + GM_K);
#pragma unroll
    for (int ks = 0; ks < GM_K; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[MI], bf[NJ];
#pragma unroll
      for (int i = 0; i < MI; i++) af[i] = sA[kr][wr * 16 * MI + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < NJ; j++) bf[j] = sB[kr][wc * 16 * NJ + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < MI; i++)
#pragma unroll
        for (int j = 0; j < NJ; j++)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      if (++steps == kc4) {
        steps = 0;
#pragma unroll
        for (int i = 0; i < MI; i++)
#pragma unroll
          for (int j = 0; j < NJ; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) acc[i][j][r] = mod_c(acc[i][j][r], p, pinv);
      }
    }
    __syncthreads();
  }
  // the old values of C, all loads at once (clamped; unused for op 2, 3)
  int32_t cold[MI][NJ][4];
#pragma unroll
  for (int i = 0; i < MI; i++)
#pragma unroll
    for (int j = 0; j < NJ; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int gr = row0 + wr * 16 * MI + i * 16 + (lane >> 4) + 4 * r;
        const int gc = col0 + wc * 16 * NJ + j * 16 + (lane & 15);
        cold[i][j][r] = Cg[(int64_t)min(gr, M - 1) * ldw + min(gc, N - 1)];
      }
#pragma unroll
  for (int i = 0; i < MI; i++)
#pragma unroll
    for (int j = 0; j < NJ; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int gr = row0 + wr * 16 * MI + i * 16 + (lane >> 4) + 4 * r;
        const int gc = col0 + wc * 16 * NJ + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          const double s = mod_c(acc[i][j][r], p, pinv);
          const double c0 = (double)cold[i][j][r];
          const double v = op == 0 ? c0 - s : op == 1 ? c0 + s : op == 2 ? s : -s;
          Cg[(int64_t)gr * ldw + gc] = (int32_t)mod_c(v, p, pinv);
        }
      }
}

// The 32 x 32 inverses of the diagonal blocks of U (panel-major, panel q at
// rows and columns [32 q, 32 q + pb)) into the diagonal of an n x n region.
__global__ void k_place_diag(int32_t* __restrict__ W, int64_t slab, int64_t ldw, int64_t offV,
                             int n, const int32_t* __restrict__ uinv, int nitems) {
  const int q = blockIdx.x, z = blockIdx.y, r = threadIdx.x >> 5, cc = threadIdx.x & 31;
  int32_t* Wz = W + (int64_t)z * slab;
  const int32_t* u = uinv + ((int64_t)q * nitems + z) * 1024;
  for (int rr = r; rr < 32; rr += blockDim.x >> 5) {
    const int gr = 32 * q + rr, gc = 32 * q + cc;
    if (gr < n && gc < n) Wz[offV + (int64_t)gr * ldw + gc] = u[rr * 32 + cc];
  }
}

// ------------------------------------------------------------------ fused LU step update
// One step of the right-looking LU after the panel [j0, j0 + pb) (pb <= 32),
// on the trailing block A22 = rows [j0 + pb, j0 + pb + M) x columns
// [j0 + pb, j0 + pb + N) of every item, in one launch:
//   U12 = L11^{-1} A12 for the workgroup's 64 columns (every workgroup of a
//   column tile computes it from A12), then A22 -= L21 U12 on its 64 x 64
//   tile; eight waves, two a SIMD, each a 32 x 16 block of the update.
// A12 stays in place until every workgroup of its column tile has read it:
// with cnt != null each workgroup counts its read (after the loads have
// completed) and the last one stores U12 over A12; without it U12 is not
// kept (a determinant needs only the diagonal).  The panel's row swaps must
// already be applied to these columns.  Sums are reduced every kc4 MFMA
// k-steps (exact chunking).
// With Uinv != null the panel factored only the pb x pb diagonal block (no
// pivot search below it) and the rows below still hold A21: every workgroup
// forms its rows' multipliers L21 = A21 U11^{-1} first (U11^{-1} from the
// panel, dense ldt x ldt per item); they are not stored (neither a
// determinant nor the inverse from [A | I] reads L).
// With next.pb > 0 the workgroup of tile (0, 0), which holds the next
// diagonal block once its own update is stored, factors that block as
// k_diag_block would (its L11^{-1}, U11^{-1} into next.Linv, next.Uinv, which
// must not be the buffers this launch reads), so the next step needs no
// launch of its own for it.
struct NextDiag {
  int pb;
  int32_t* Linv;
  int32_t* Uinv;
  int32_t* piv;
  int64_t piv_stride;
  int32_t* flags;
};

__global__ __launch_bounds__(512) void k_lu_update(int32_t* __restrict__ W, int64_t slab,
                                                   int64_t ldw, int j0, int pb, int M, int N,
                                                   const int32_t* __restrict__ Linv, int ldt,
                                                   const int32_t* __restrict__ Uinv,
                                                   const Modulus* __restrict__ mods, int kc4,
                                                   unsigned* __restrict__ cnt, int cnt_stride,
                                                   NextDiag next) {
  constexpr int T = 512;                                // eight waves, two a SIMD
  // Workgroup order: tile (0, 0) of every item first (the tile whose
  // workgroup factors the next diagonal block, the head of the critical
  // path), then the other tiles item by item.
  const int tx = gridDim.x, ty = gridDim.y;
  const int L = blockIdx.x + tx * (blockIdx.y + ty * blockIdx.z);
  int z = L, bx = 0, by = 0;
  if (L >= (int)gridDim.z) {
    const int per = tx * ty - 1, L2 = L - gridDim.z;
    z = L2 / per;
    const int tt = 1 + L2 % per;
    bx = tt % tx;
    by = tt / tx;
  }
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 2, wc = wave & 3;              // update: a 32 x 16 block a wave
  const double p = mods[z].p, pinv = mods[z].pinv;
  int32_t* Wz = W + (int64_t)z * slab;
  const int r0 = j0 + pb;                               // first row and column of A22
  const int row0 = by * GB_M, col0 = bx * GB_N;
  __shared__ double sA[GB_K][GB_M + 2];                 // L21 tile, k-major
  __shared__ double sB[GB_K][GB_N + 2];                 // A12 tile, then U12
  __shared__ double sT[32][33];                         // L11^{-1}
  __shared__ double sU[32][33];                         // U11^{-1} (no-pivot mode)
  __shared__ int s_last;
  // All loads at once: L11^{-1}, U11^{-1}, A12, L21 and the old values of
  // the tile.  Every load is unconditional, from an index clamped into the
  // valid range (M, N, pb >= 1), and the padding is selected afterwards: a
  // load under a condition becomes a branch that waits for its own data.
  const int32_t* Tz = Linv + (int64_t)z * ldt * ldt;
  const int32_t* Uz = Uinv != nullptr ? Uinv + (int64_t)z * ldt * ldt : Tz;
  int32_t vt[1024 / T], vu[1024 / T];
#pragma unroll
  for (int u = 0; u < 1024 / T; u++) {
    const int e = u * T + t, r = min(e >> 5, pb - 1), c = min(e & 31, pb - 1);
    vt[u] = Tz[r * ldt + c];
    vu[u] = Uz[r * ldt + c];
  }
  int32_t va[GB_M * GB_K / T], vb[GB_K * GB_N / T], vc[2][4];
#pragma unroll
  for (int u = 0; u < GB_M * GB_K / T; u++) {
    const int f = u * T + t, r = f / GB_K, k = f % GB_K;
    va[u] = Wz[(int64_t)(r0 + min(row0 + r, M - 1)) * ldw + j0 + min(k, pb - 1)];
  }
#pragma unroll
  for (int u = 0; u < GB_K * GB_N / T; u++) {
    const int f = u * T + t, k = f / GB_N, c = f % GB_N;
    vb[u] = Wz[(int64_t)(j0 + min(k, pb - 1)) * ldw + r0 + min(col0 + c, N - 1)];
  }
  const int gc = col0 + wc * 16 + (lane & 15);
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int gr = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
      vc[i][r] = Wz[(int64_t)(r0 + min(gr, M - 1)) * ldw + r0 + min(gc, N - 1)];
    }
#pragma unroll
  for (int u = 0; u < 1024 / T; u++) {
    const int e = u * T + t, r = e >> 5, c = e & 31;
    const bool in = r < pb && c < pb;
    // L11^{-1} is unit lower triangular: only its entries below the
    // diagonal are read (the diagonal block's factorisation stores no others)
    sT[r][c] = in ? (c < r ? (double)vt[u] : (c == r ? 1.0 : 0.0)) : 0.0;
    sU[r][c] = in ? (double)vu[u] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < GB_M * GB_K / T; u++) {
    const int f = u * T + t, r = f / GB_K, k = f % GB_K;
    sA[k][r] = (row0 + r < M && k < pb) ? (double)va[u] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < GB_K * GB_N / T; u++) {
    const int f = u * T + t, k = f / GB_N, c = f % GB_N;
    sB[k][c] = (k < pb && col0 + c < N) ? (double)vb[u] : 0.0;
  }
  __syncthreads();
  if (Uinv != nullptr) {
    // L21 = A21 U11^{-1} (64 x 32): one 16 x 16 MFMA block a wave (rows
    // 16 (w >> 1), columns 16 (w & 1)); written back into sA (k-major) after
    // every wave has read A21
    const int lr = (wave >> 1) * 16, lc = (wave & 1) * 16;
    v4d l2 = (v4d){0.0, 0.0, 0.0, 0.0};
    int steps = 0;
#pragma unroll
    for (int ks = 0; ks < 32; ks += 4) {
      const int kr = ks + (lane >> 4);
      l2 = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[kr][lr + (lane & 15)], sU[kr][lc + (lane & 15)],
                                               l2, 0, 0, 0);
      if (++steps == kc4) {
        steps = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) l2[r] = mod_c(l2[r], p, pinv);
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; r++) sA[lc + (lane & 15)][lr + (lane >> 4) + 4 * r] = mod_c(l2[r], p, pinv);
    __syncthreads();
  }
  // U12 = L11^{-1} A12 (32 x 64): one 16 x 16 MFMA block a wave (rows
  // 16 (w >> 2), columns 16 (w & 3))
  const int ur = (wave >> 2) * 16, uc = (wave & 3) * 16;
  v4d u2 = (v4d){0.0, 0.0, 0.0, 0.0};
  {
    int steps = 0;
#pragma unroll
    for (int ks = 0; ks < 32; ks += 4) {
      const int kr = ks + (lane >> 4);
      u2 = __builtin_amdgcn_mfma_f64_16x16x4f64(sT[ur + (lane & 15)][kr], sB[kr][uc + (lane & 15)],
                                               u2, 0, 0, 0);
      if (++steps == kc4) {
        steps = 0;
#pragma unroll
        for (int r = 0; r < 4; r++) u2[r] = mod_c(u2[r], p, pinv);
      }
    }
  }
  __syncthreads();                                      // every wave is done with A12
#pragma unroll
  for (int r = 0; r < 4; r++) sB[ur + (lane >> 4) + 4 * r][uc + (lane & 15)] = mod_c(u2[r], p, pinv);
  if (cnt != nullptr && t == 0) {
    const unsigned prev = atomicAdd(cnt + (int64_t)z * cnt_stride + bx, 1u);
    s_last = prev + 1 == (unsigned)ty;
  }
  __syncthreads();
  if (cnt != nullptr && s_last) {                       // the last reader stores U12
    for (int e = t; e < 32 * GB_N; e += T) {
      const int k = e / GB_N, c = e % GB_N;
      if (k < pb && col0 + c < N) Wz[(int64_t)(j0 + k) * ldw + r0 + col0 + c] = (int32_t)sB[k][c];
    }
  }
  // A22 -= L21 U12: wave (wr, wc) the 32 x 16 block at rows 32 wr, columns 16 wc
  v4d acc[2];
  acc[0] = acc[1] = (v4d){0.0, 0.0, 0.0, 0.0};
  int steps = 0;
#pragma unroll
  for (int ks = 0; ks < GB_K; ks += 4) {
    const int kr = ks + (lane >> 4);
    const double bf = sB[kr][wc * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 2; i++)
      acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[kr][wr * 32 + i * 16 + (lane & 15)], bf,
                                                   acc[i], 0, 0, 0);
    if (++steps == kc4) {
      steps = 0;
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int r = 0; r < 4; r++) acc[i][r] = mod_c(acc[i][r], p, pinv);
    }
  }
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int gr = row0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
      if (gr < M && gc < N)
        Wz[(int64_t)(r0 + gr) * ldw + r0 + gc] =
            (int32_t)mod_c((double)vc[i][r] - mod_c(acc[i][r], p, pinv), p, pinv);
    }
  if (next.pb > 0 && bx == 0 && by == 0) {
    __syncthreads();                                    // the tile is stored
    diag_block_body(Wz + (int64_t)r0 * ldw + r0, ldw, next.pb, p, pinv,
                    next.piv + (int64_t)z * next.piv_stride, r0, next.flags + z,
                    next.Linv + (int64_t)z * 1024, next.Uinv + (int64_t)z * 1024);
  }
}

// ------------------------------------------------------------------ K4: in-place triangular apply
// X <- Tinv[z] * X for the strip X = rows [r0, r0+kb) x columns [c0, c0+N)
// of every item (U12 = L11^{-1} A12, or X_blk = U11^{-1} Y_blk).  A
// workgroup loads its whole kb x 64 column strip into LDS before it writes,
// so the update in place is safe (no other workgroup touches those columns).
// With sw_pb > 0 the workgroup first applies the row swaps of the panel
// [sw_j0, sw_j0 + sw_pb) (row sw_j0+j <-> piv[sw_j0+j], in order) to its
// columns, so a separate swap launch is not needed.
__global__ __launch_bounds__(256) void k_trsm_apply(int32_t* __restrict__ W, int64_t slab,
                                                    int64_t ldw, int r0, int kb, int c0, int N,
                                                    const int32_t* __restrict__ Tinv, int ldt,
                                                    const Modulus* __restrict__ mods, int kc4,
                                                    const int32_t* __restrict__ piv,
                                                    int64_t piv_stride, int sw_j0, int sw_pb) {
  const int z = blockIdx.y;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const double p = mods[z].p, pinv = mods[z].pinv;
  int32_t* Xg = W + (int64_t)z * slab + (int64_t)r0 * ldw + c0;
  const int32_t* Tz = Tinv + (int64_t)z * ldt * ldt;
  const int col0 = blockIdx.x * GB_N;
  if (sw_pb > 0) {
    const int32_t* pz = piv + (int64_t)z * piv_stride + sw_j0;
    // one pivot a thread (a loop over them would wait for each load in turn)
    const bool any = __syncthreads_or(t < sw_pb && pz[t] != sw_j0 + t);
    if (any) {                                   // uniform across the workgroup
      int32_t* Wc = W + (int64_t)z * slab + c0;
      if (t < GB_N && col0 + t < N) {
        const int gc = col0 + t;
        for (int j = 0; j < sw_pb; j++) {
          const int rw = pz[j];
          if (rw != sw_j0 + j) {
            const int32_t v = Wc[(int64_t)(sw_j0 + j) * ldw + gc];
            Wc[(int64_t)(sw_j0 + j) * ldw + gc] = Wc[(int64_t)rw * ldw + gc];
            Wc[(int64_t)rw * ldw + gc] = v;
          }
        }
      }
      __syncthreads();
    }
  }
  extern __shared__ double sX[];             // [ldt][GB_N + 2], then Tinv when ldt <= 32
  constexpr int LDX = GB_N + 2;
  const bool stage_t = ldt <= 32;              // the inverse in LDS, not read per k-step
  double* sT = sX + ldt * LDX;
  for (int e = t; e < ldt * GB_N; e += 256) {
    const int k = e / GB_N, c = e % GB_N;
    const int gc = col0 + c;
    sX[k * LDX + c] = (k < kb && gc < N) ? (double)Xg[(int64_t)k * ldw + gc] : 0.0;
  }
  if (stage_t)
    for (int e = t; e < ldt * ldt; e += 256) sT[e] = (double)Tz[e];
  __syncthreads();
  for (int rb = 0; rb < kb; rb += GB_M) {
    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};
    int steps = 0;
    for (int ks = 0; ks < kb; ks += 4) {
      const int kr = ks + (lane >> 4);
      double af[2], bf[2];
#pragma unroll
      for (int i = 0; i < 2; i++) {
        const int rr = rb + wr * 32 + i * 16 + (lane & 15);
        af[i] = (rr < kb && kr < kb) ? (stage_t ? sT[rr * ldt + kr] : (double)Tz[rr * ldt + kr])
                                     : 0.0;
      }
#pragma unroll
      for (int j = 0; j < 2; j++) bf[j] = sX[kr * LDX + wc * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      if (++steps == kc4) {
        steps = 0;
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) acc[i][j][r] = mod_c(acc[i][j][r], p, pinv);
      }
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) {
          const int gr = rb + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
          const int gc = col0 + wc * 32 + j * 16 + (lane & 15);
          if (gr < kb && gc < N) Xg[(int64_t)gr * ldw + gc] = (int32_t)mod_c(acc[i][j][r], p, pinv);
        }
  }
}

// ------------------------------------------------------------------ int8 limb path
// Centred residues |r| < 2^22 (p < 2^23) in three balanced signed limbs
// (limb_word, i8tile.hpp).

// Limb planes of an M x K block (A: row-major, k contiguous) or of a K x N
// block stored transposed (B: column j's K values contiguous), both padded
// with zeros to Rp x Kp (multiples of 64).  Out: P[z][3][Rp][Kp].  One
// 64 x 64 tile a workgroup: the int32 tile is read row by row into LDS, and
// each thread packs byte j of four consecutive k values into one word of
// plane j (v_perm_b32), so reads and writes are both contiguous.
__global__ __launch_bounds__(256) void k_split(const int32_t* __restrict__ W, int64_t slab,
                                               int64_t off, int64_t ldw, int rows, int K, int Kp,
                                               int64_t Rp, int transpose, int8_t* __restrict__ P,
                                               int64_t pslab) {
  __shared__ uint32_t sT[64][65];
  const int z = blockIdx.z;
  const int32_t* Wz = W + (int64_t)z * slab + off;
  limb_split_tile([&](int r, int c) { return Wz[(int64_t)r * ldw + c]; }, rows, K, Kp, Rp,
                  transpose, P + (int64_t)z * pslab, sT);
}

// C[z] = (C[z] - A[z] B[z]) mod p_z with A, B given as limb planes (Rp x Kp,
// zero-padded, so every load is in range and unconditional).
// C_s = sum_{a+b=s} A_a B_b on v_mfma_i32_16x16x64_i8 (exact while
// 3 K 2^14 < 2^31), then C -= sum_s (C_s mod p)(2^(8s) mod p) mod p in FP64.
// The next K chunk's loads are in flight during this chunk's products.
// Lane l supplies A[l%16][16(l/16) .. +16) and B^T[l%16][same k]; result
// element r of lane l is D[4(l/16) + r][l%16].

__global__ __launch_bounds__(256) void k_gemm_i8(int32_t* __restrict__ W, int64_t slab,
                                                 int64_t offC, int64_t ldw, int M, int N,
                                                 const int8_t* __restrict__ PA,
                                                 const int8_t* __restrict__ PB, int64_t pslabA,
                                                 int64_t pslabB, int64_t MpA, int64_t NpB, int Kp,
                                                 const Modulus* __restrict__ mods) {
  const int z = blockIdx.z;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const double p = mods[z].p, pinv = mods[z].pinv;
  const int row0 = blockIdx.y * GB_M, col0 = blockIdx.x * GB_N;
  const int8_t* Az = PA + (int64_t)z * pslabA;
  const int8_t* Bz = PB + (int64_t)z * pslabB;
  __shared__ __attribute__((aligned(16))) int8_t sA[3][I8_TILE][I8_LD];
  __shared__ __attribute__((aligned(16))) int8_t sB[3][I8_TILE][I8_LD];
  v4i_t acc[5][2][2];
  i8_tile_product(Az, Bz, MpA * Kp, NpB * Kp, Kp, row0, col0, sA, sB, acc);
  // weights 2^(8s) mod p, centred
  double wgt[5];
  wgt[0] = 1.0;
#pragma unroll
  for (int s = 1; s < 5; s++) wgt[s] = mod_c(wgt[s - 1] * 256.0, p, pinv);
  int32_t* Cg = W + (int64_t)z * slab + offC;
  int32_t cold[2][2][4];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int gr = row0 + wr * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int gc = col0 + wc * 32 + j * 16 + (lane & 15);
        cold[i][j][r] = Cg[(int64_t)min(gr, M - 1) * ldw + min(gc, N - 1)];
      }
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int gr = row0 + wr * 32 + i * 16 + 4 * (lane >> 4) + r;
        const int gc = col0 + wc * 32 + j * 16 + (lane & 15);
        if (gr < M && gc < N) {
          double v = 0.0;
#pragma unroll
          for (int s = 0; s < 5; s++) v += mod_c((double)acc[s][i][j][r], p, pinv) * wgt[s];
          v = mod_c(v, p, pinv);
          Cg[(int64_t)gr * ldw + gc] = (int32_t)mod_c((double)cold[i][j][r] - v, p, pinv);
        }
      }
}

// ------------------------------------------------------------------ K6: determinant
// det mod p = (-1)^(#swaps) * prod u_jj, canonical; 0 if flagged singular.
__global__ __launch_bounds__(256) void k_det_finalize(const int32_t* __restrict__ W, int64_t ldw,
                                                      int64_t slab, int n,
                                                      const int32_t* __restrict__ piv,
                                                      int64_t piv_stride,
                                                      const int32_t* __restrict__ flags,
                                                      const Modulus* __restrict__ mods,
                                                      uint32_t* __restrict__ out) {
  const int z = blockIdx.x;
  const int t = threadIdx.x;
  const double p = mods[z].p, pinv = mods[z].pinv;
  const int32_t* Wz = W + (int64_t)z * slab;
  double prod = 1.0;
  int swaps = 0;
  for (int j = t; j < n; j += 256) {
    prod = mul_mod(prod, (double)Wz[(int64_t)j * ldw + j], p, pinv);
    swaps += piv[(int64_t)z * piv_stride + j] != j;
  }
  __shared__ double sp[256];
  __shared__ int ss[256];
  sp[t] = prod;
  ss[t] = swaps;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      sp[t] = mul_mod(sp[t], sp[t + s], p, pinv);
      ss[t] += ss[t + s];
    }
    __syncthreads();
  }
  if (t == 0) {
    double d = sp[0];
    if (ss[0] & 1) d = -d;
    if (flags[z]) d = 0.0;
    out[z] = to_canonical(d, p);
  }
}

// ------------------------------------------------------------------ inverse extraction
// Cu[i][j] = canonical residue of W[z=0][i][n + j] (the right half of [A | I]
// after elimination and back substitution holds A^{-1} mod p).
__global__ void k_extract_inverse(const int32_t* __restrict__ W, int64_t slab, int64_t ldw,
                                  int64_t col0, int n, const Modulus* __restrict__ mods,
                                  uint32_t* __restrict__ Cu) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y, z = blockIdx.z;
  if (j >= n || i >= n) return;
  const double p = mods[z].p;
  Cu[((int64_t)z * n + i) * n + j] =
      to_canonical((double)W[(int64_t)z * slab + (int64_t)i * ldw + col0 + j], p);
}

// ------------------------------------------------------------------ A packing and norms
// Ai = A as int32 (the entry bound |a_ij| < 2^31 is checked on the host).
__global__ void k_pack_i32(const int64_t* __restrict__ A, int64_t lda, int n,
                           int32_t* __restrict__ Ai) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n || i >= n) return;
  Ai[(int64_t)i * n + j] = (int32_t)A[(int64_t)i * lda + j];
}

// out[j] = sum_i a_ij^2 (columns), out[n + i] = sum_j a_ij^2 (rows), both in
// FP64 (rounded; the host adds a relative margin), and amax[j] = max_i |a_ij|.
// Squared column norms and column maxima: 64 columns per workgroup, the 16
// waves take interleaved rows and combine through LDS.
__global__ __launch_bounds__(1024) void k_col_norms(const int64_t* __restrict__ A, int64_t lda,
                                                    int n, double* __restrict__ out,
                                                    double* __restrict__ amax) {
  __shared__ double s_s[16][65];
  __shared__ double s_m[16][65];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  double s = 0.0, m = 0.0;
  if (j < n) {
    for (int i = g; i < n; i += 16) {
      const double a = (double)A[(int64_t)i * lda + j];
      s = fma(a, a, s);
      m = fmax(m, fabs(a));
    }
  }
  s_s[g][lane] = s;
  s_m[g][lane] = m;
  __syncthreads();
  if (g == 0 && j < n) {
    for (int w = 1; w < 16; w++) {
      s += s_s[w][lane];
      m = fmax(m, s_m[w][lane]);
    }
    out[j] = s;
    amax[j] = m;
  }
}
__global__ __launch_bounds__(256) void k_row_norms(const int64_t* __restrict__ A, int64_t lda,
                                                   int n, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) {
    const double a = (double)A[(int64_t)i * lda + j];
    s = fma(a, a, s);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) out[n + i] = s;
}

// The same sums over the whole chip: workgroup (x, y) takes the 64 columns
// [64x, 64x + 64) of the 64 rows [64y, 64y + 64) (a wave 16 rows, a lane a
// column) and writes its partial column sums and maxima (part[y][j],
// part[Y + y][j], Y = gridDim.y) and partial row sums (part[2Y + x][i]);
// k_norm_finish adds the partials of each column and row in a fixed order,
// so the bounds do not depend on the schedule.
__global__ __launch_bounds__(256) void k_norm_part(const int64_t* __restrict__ A, int64_t lda,
                                                   int n, double* __restrict__ part) {
  __shared__ double s_s[4][64];
  __shared__ double s_m[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  const int Y = gridDim.y;
  double* const rowp = part + (size_t)(2 * Y + blockIdx.x) * n;
  double s = 0.0, m = 0.0;
  const int i0 = blockIdx.y * 64 + wv * 16;
  double a[16];
#pragma unroll
  for (int r = 0; r < 16; r++) {
    const int i = i0 + r;
    a[r] = (i < n && j < n) ? (double)A[(int64_t)i * lda + j] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < 16; r++) {
    s = fma(a[r], a[r], s);
    m = fmax(m, fabs(a[r]));
    double rs = a[r] * a[r];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rs += __shfl_xor(rs, off, 64);
    if (lane == 0 && i0 + r < n) rowp[i0 + r] = rs;
  }
  s_s[wv][lane] = s;
  s_m[wv][lane] = m;
  __syncthreads();
  if (wv == 0 && j < n) {
    part[(size_t)blockIdx.y * n + j] = ((s_s[0][lane] + s_s[1][lane]) + s_s[2][lane]) + s_s[3][lane];
    part[(size_t)(Y + blockIdx.y) * n + j] =
        fmax(fmax(s_m[0][lane], s_m[1][lane]), fmax(s_m[2][lane], s_m[3][lane]));
  }
}

// Thread t < n: column t's sum and maximum over the Y row chunks; thread
// n + i: row i's sum over the X column strips.
__global__ __launch_bounds__(256) void k_norm_finish(const double* __restrict__ part, int n, int X,
                                                     int Y, double* __restrict__ out2n,
                                                     double* __restrict__ amax) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < n) {
    double s = 0.0, m = 0.0;
    for (int y = 0; y < Y; y++) {
      s += part[(size_t)y * n + t];
      m = fmax(m, part[(size_t)(Y + y) * n + t]);
    }
    out2n[t] = s;
    amax[t] = m;
  } else if (t < 2 * n) {
    const int i = t - n;
    double s = 0.0;
    for (int x = 0; x < X; x++) s += part[(size_t)(2 * Y + x) * n + i];
    out2n[n + i] = s;
  }
}

// ------------------------------------------------------------------ launchers
#define LAUNCH_CHECK() do { hipError_t e_ = hipGetLastError(); if (e_ != hipSuccess) return e_; } while (0)

hipError_t launch_residues(const int64_t* A, int64_t lda, int n, int ncols, int32_t* W, int64_t ldw,
                           int64_t slab, const Modulus* mods, int nitems, hipStream_t st) {
  if (n <= 0 || ncols <= 0) return hipSuccess;
  dim3 grid((ncols + 255) / 256, n);
  k_residues<<<grid, 256, 0, st>>>(A, lda, n, ncols, W, ldw, slab, mods, nitems);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_panel(int32_t* W, int64_t ldw, int64_t slab, int n, int j0, int pb, int pbw,
                        const Modulus* mods, int32_t* piv, int64_t piv_stride, int32_t* flags,
                        int32_t* Linv, int32_t* Uinv, int kc, int nitems, int ncols_sw,
                        hipStream_t st) {
  const int m = n - j0;
  // the kernel reduces every 8 columns: exact when kc >= 8 (all p < 2^26)
  if (pb > pbw || pb > m || kc < 8) return hipErrorInvalidValue;
  if (pbw == 32 && m <= 1024)
    k_panel<32, 2><<<nitems, 512, 0, st>>>(W, ldw, slab, n, j0, pb, mods, piv, piv_stride, flags, Linv, Uinv, ncols_sw);
  else if (pbw == 16 && m <= 2048)
    k_panel<16, 4><<<nitems, 512, 0, st>>>(W, ldw, slab, n, j0, pb, mods, piv, piv_stride, flags, Linv, Uinv, ncols_sw);
  else if (pbw == 8 && m <= 4096)
    k_panel<8, 8><<<nitems, 512, 0, st>>>(W, ldw, slab, n, j0, pb, mods, piv, piv_stride, flags, Linv, Uinv, ncols_sw);
  else
    return hipErrorInvalidValue;
  LAUNCH_CHECK();
  return hipSuccess;
}

// Panel width for a panel whose first row is j0: its m = n - j0 rows must
// fit the 1024 threads times the rows each holds (and m x width <= 32768).
int panel_width_for(int m) { return m <= 1024 ? 32 : (m <= 2048 ? 16 : 8); }

hipError_t launch_diag_block(int32_t* W, int64_t ldw, int64_t slab, int j0, int pb,
                             const Modulus* mods, int32_t* piv, int64_t piv_stride, int32_t* flags,
                             int32_t* Linv, int32_t* Uinv, int nitems, hipStream_t st) {
  if (pb < 1 || pb > 32 || !Linv || !Uinv) return hipErrorInvalidValue;
  k_diag_block<<<nitems, 128, 0, st>>>(W, ldw, slab, j0, pb, mods, piv, piv_stride, flags, Linv, Uinv);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_swaps(int32_t* W, int64_t ldw, int64_t slab, int j0, int pb, const int32_t* piv,
                        int64_t piv_stride, int c0a, int c1a, int c0b, int c1b, int nitems,
                        hipStream_t st) {
  const int w = (c1a - c0a) + (c1b - c0b);
  if (w <= 0) return hipSuccess;
  dim3 grid((w + 255) / 256, nitems);
  k_swaps<<<grid, 256, 0, st>>>(W, ldw, slab, j0, pb, piv, piv_stride, c0a, c1a, c0b, c1b);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_tri_inv(const int32_t* W, int64_t ldw, int64_t slab, int k0, int kb,
                          const Modulus* mods, int32_t* Tinv, int ldt, int nitems, hipStream_t st) {
  if (kb <= 0) return hipSuccess;
  if (kb > ldt || ldt > 128) return hipErrorInvalidValue;
  k_tri_inv<<<nitems, 1024, 0, st>>>(W, ldw, slab, k0, kb, mods, Tinv, ldt);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_trsm_apply(int32_t* W, int64_t slab, int64_t ldw, int r0, int kb, int c0, int N,
                             const int32_t* Tinv, int ldt, const Modulus* mods, int kc4,
                             const int32_t* piv, int64_t piv_stride, int sw_j0, int sw_pb,
                             int nitems, hipStream_t st) {
  if (kb <= 0 || N <= 0) return hipSuccess;
  if (kb > ldt || (ldt % 4) != 0) return hipErrorInvalidValue;
  dim3 grid((N + GB_N - 1) / GB_N, nitems);
  const size_t sh = ((size_t)ldt * (GB_N + 2) + (ldt <= 32 ? (size_t)ldt * ldt : 0)) * sizeof(double);
  k_trsm_apply<<<grid, 256, sh, st>>>(W, slab, ldw, r0, kb, c0, N, Tinv, ldt, mods, kc4, piv,
                                      piv_stride, sw_j0, sw_pb);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_gemm_f64(int32_t* W, int64_t slab, int64_t offC, int64_t offA, int64_t offB,
                           int64_t ldw, int M, int N, int K, const Modulus* mods, int kc4,
                           int nitems, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  return launch_gemm_mod(W, slab, offC, offA, offB, ldw, M, N, K, mods, kc4, 0, false, nitems, st);
}

hipError_t launch_lu_update(int32_t* W, int64_t slab, int64_t ldw, int j0, int pb, int M, int N,
                            const int32_t* Linv, int ldt, const int32_t* Uinv,
                            const Modulus* mods, int kc4, unsigned* cnt, int cnt_stride,
                            int nitems, hipStream_t st, int next_pb, int32_t* next_Linv,
                            int32_t* next_Uinv, int32_t* piv, int64_t piv_stride, int32_t* flags) {
  if (M < 0 || N <= 0 || nitems <= 0) return hipSuccess;
  if (pb < 1 || pb > 32 || pb > ldt || kc4 < 1) return hipErrorInvalidValue;
  dim3 grid((N + GB_N - 1) / GB_N, std::max(1, (M + GB_M - 1) / GB_M), nitems);
  if (cnt != nullptr && (int)grid.x > cnt_stride) return hipErrorInvalidValue;
  if (next_pb > 0 && (next_pb > 32 || next_pb > M || !next_Linv || !next_Uinv || !piv || !flags ||
                      next_Linv == Linv || next_Uinv == Uinv))
    return hipErrorInvalidValue;
  const NextDiag nd{next_pb, next_Linv, next_Uinv, piv, piv_stride, flags};
  k_lu_update<<<grid, 512, 0, st>>>(W, slab, ldw, j0, pb, M, N, Linv, ldt, Uinv, mods, kc4, cnt,
                                    cnt_stride, nd);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_gemm_mod(int32_t* W, int64_t slab, int64_t offC, int64_t offA, int64_t offB,
                           int64_t ldw, int M, int N, int K, const Modulus* mods, int kc4, int op,
                           bool upper_a, int nitems, hipStream_t st, int nouter,
                           int64_t slab_outer, bool mod_by_outer) {
  if (M <= 0 || N <= 0 || nitems <= 0 || nouter <= 0) return hipSuccess;
  if (op < 0 || op > 3 || kc4 < 1 || (int64_t)nitems * nouter > 65535) return hipErrorInvalidValue;
  dim3 grid((N + 63) / 64, (M + 63) / 64, nitems * nouter);
  // eight waves of 32 x 16 (two a SIMD hide each other's LDS and MFMA
  // latencies): 1.28x the four-wave form on the 570-prime trailing updates
  k_gemm_mod<2, 4, 2, 1><<<grid, 512, 0, st>>>(W, slab, offC, offA, offB, ldw, M, N, K, mods,
                                               kc4, op, upper_a ? 1 : 0, nitems, slab_outer,
                                               mod_by_outer ? 1 : 0);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_place_diag(int32_t* W, int64_t slab, int64_t ldw, int64_t offV, int n,
                             const int32_t* uinv, int nitems, hipStream_t st) {
  if (n <= 0 || nitems <= 0) return hipSuccess;
  k_place_diag<<<dim3((n + 31) / 32, nitems), 256, 0, st>>>(W, slab, ldw, offV, n, uinv, nitems);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_split(const int32_t* W, int64_t slab, int64_t off, int64_t ldw, int rows, int K,
                        int Kp, int64_t Rp, int transpose, int8_t* P, int64_t pslab, int nitems,
                        hipStream_t st) {
  if (rows <= 0 || K <= 0 || nitems <= 0) return hipSuccess;
  if (Kp % 64 || Rp % 64 || Kp < K || Rp < rows) return hipErrorInvalidValue;
  dim3 grid(Kp / 64, (unsigned)(Rp / 64), nitems);
  k_split<<<grid, 256, 0, st>>>(W, slab, off, ldw, rows, K, Kp, Rp, transpose, P, pslab);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_gemm_i8(int32_t* W, int64_t slab, int64_t offC, int64_t ldw, int M, int N,
                          const int8_t* PA, const int8_t* PB, int64_t pslabA, int64_t pslabB,
                          int64_t MpA, int64_t NpB, int Kp, const Modulus* mods, int nitems,
                          hipStream_t st) {
  if (M <= 0 || N <= 0 || Kp <= 0 || nitems <= 0) return hipSuccess;
  if (Kp % I8_K || MpA % GB_M || NpB % GB_N || MpA < M || NpB < N || Kp > 43690)
    return hipErrorInvalidValue;
  dim3 grid((N + GB_N - 1) / GB_N, (M + GB_M - 1) / GB_M, nitems);
  k_gemm_i8<<<grid, 256, 0, st>>>(W, slab, offC, ldw, M, N, PA, PB, pslabA, pslabB, MpA, NpB, Kp,
                                  mods);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_det_finalize(const int32_t* W, int64_t ldw, int64_t slab, int n,
                               const int32_t* piv, int64_t piv_stride, const int32_t* flags,
                               const Modulus* mods, uint32_t* out, int nitems, hipStream_t st) {
  k_det_finalize<<<nitems, 256, 0, st>>>(W, ldw, slab, n, piv, piv_stride, flags, mods, out);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_extract_inverse(const int32_t* W, int64_t slab, int64_t ldw, int64_t col0, int n,
                                  const Modulus* mods, uint32_t* Cu, int nitems, hipStream_t st) {
  if (n <= 0 || nitems <= 0) return hipSuccess;
  dim3 grid((n + 255) / 256, n, nitems);
  k_extract_inverse<<<grid, 256, 0, st>>>(W, slab, ldw, col0, n, mods, Cu);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_pack_i32(const int64_t* A, int64_t lda, int n, int32_t* Ai, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 grid((n + 255) / 256, n);
  k_pack_i32<<<grid, 256, 0, st>>>(A, lda, n, Ai);
  LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t launch_norms(const int64_t* A, int64_t lda, int n, double* out2n, double* amax,
                        hipStream_t st) {
  if (n <= 0) return hipSuccess;
  k_col_norms<<<(n + 63) / 64, 1024, 0, st>>>(A, lda, n, out2n, amax);
  LAUNCH_CHECK();
  k_row_norms<<<(n + 3) / 4, 256, 0, st>>>(A, lda, n, out2n);
  LAUNCH_CHECK();
  return hipSuccess;
}

size_t norms_scratch(int n) {
  const size_t b = (size_t)(n + 63) / 64;
  return 3 * b * (size_t)n;
}

hipError_t launch_norms_wide(const int64_t* A, int64_t lda, int n, double* out2n, double* amax,
                             double* part, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int b = (n + 63) / 64;
  k_norm_part<<<dim3(b, b), 256, 0, st>>>(A, lda, n, part);
  LAUNCH_CHECK();
  k_norm_finish<<<(2 * n + 255) / 256, 256, 0, st>>>(part, n, b, b, out2n, amax);
  LAUNCH_CHECK();
  return hipSuccess;
}

// k_trsm_apply takes its strip (and a small inverse) as dynamic LDS: at most
// 128 x 66 doubles for the 128-wide outer inverses; its own static LDS (the
// workgroup vote) must fit beside it in the 160 KB of a CU.
hipError_t configure_kernels() {
  return hipFuncSetAttribute((const void*)k_trsm_apply,
                             hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
}

}  // namespace detk
