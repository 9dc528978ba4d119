// Persistent LU modulo p over a work queue of (matrix, prime) items, for
// gfx950: the batched form of the Chinese-remaindering side.
//
// Section 2.1 obtains each modular determinant from an LU factorisation
// modulo a prime, and Section 6 notes that the LU runs of one CRA step are
// independent; across a batch of matrices every (matrix, prime) pair is an
// independent item.  Here one workgroup takes one item at a time from a
// device queue (an atomic counter over an item array that the host sorts by
// decreasing order n, so the largest items start first) and factors it
// entirely on its own: residue reduction into its private slab, then per
// panel of PB columns the panel body (pivot search, row swaps, multipliers,
// in registers and LDS), U12 = L11^{-1} A12 and A22 -= L21 U12 on FP64 MFMA
// (v_mfma_f64_16x16x4f64) over 64 x 64 tiles, and finally the product of the
// pivots with the swap parity.  The grid is a fixed number of workgroups (a
// multiple of the CU count chosen by the autotuner, WPE the waves per SIMD the
// register budget allows); every workgroup leaves
// its loop once the counter passes the item count, so the grid always drains.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "modp.hpp"
#include "panel.hpp"

namespace detk {

typedef double v4d_q __attribute__((ext_vector_type(4)));

// Item of the queue (also declared for the host in kernels.hpp).
static_assert(sizeof(LuItem) == 32, "item layout");

// Per-workgroup private memory: the slab (ws_stride int32) in `ws`; in `aux`
// (aux_stride int32): the pivot record (up to RPT * 256 rows), the
// singularity flag and the panel's L11^{-1}.  Results: out[i] = det mod p of
// item i, written with a system-scope store so that the host can see each
// one as it completes when `out` is mapped host memory (the host fills it
// with 0xFFFFFFFF, which no residue equals, before the launch).
template <int PB, int RPT, int WPE>
__global__ __launch_bounds__(256, WPE) void k_lu_queue(const LuItem* __restrict__ items, int nitems,
                                                       unsigned* __restrict__ next,
                                                       int32_t* __restrict__ ws, int64_t ws_stride,
                                                       int32_t* __restrict__ aux, int64_t aux_stride,
                                                       uint32_t* __restrict__ out) {
  constexpr int T = 256, MROWS = RPT * T, SP = PB + 1;
  constexpr int SW = MROWS + 4;                 // row stride of the U12 strip (int32)
  __shared__ int32_t sP[MROWS * SP];            // the finished panel (L21 read from here)
  __shared__ __attribute__((aligned(16))) int32_t sS[PB * SW];   // A12, then U12 (all columns)
  __shared__ double sT[PB][PB + 1];             // L11^{-1}
  __shared__ int s_item;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  int32_t* W = ws + (int64_t)blockIdx.x * ws_stride;
  int32_t* piv = aux + (int64_t)blockIdx.x * aux_stride;
  int32_t* flag = piv + MROWS;
  int32_t* linv = flag + 4;
  for (;;) {
    if (t == 0) s_item = (int)atomicAdd(next, 1u);
    __syncthreads();
    const int it = s_item;
    __syncthreads();                             // every thread has read s_item
    if (it >= nitems) break;
    const LuItem I = items[it];
    const int n = I.n;
    const int64_t ldw = (int64_t)((n + 63) / 64 * 64 + 4);
    const double p = (double)I.p, pinv = 1.0 / p;
    // exact chunk of FP64 sums of centred products: K h^2 + h <= 2^53
    const double h = (double)((I.p - 1) / 2);
    const int kc = (int)fmin(floor((9007199254740992.0 - h) / (h * h)), 1e6);
    const int kc4 = kc >= 8 ? kc / 4 : 1;
    // residue reduction (K1) into the slab: wave w takes rows w, w + 4, ...,
    // lane l columns l + 64 u; eight loads in flight a lane
    for (int i = wave; i < n; i += 4) {
      const int64_t* row = I.A + (int64_t)i * I.lda;
      int32_t* wrow = W + (int64_t)i * ldw;
      int64_t v[8];
#pragma unroll
      for (int u = 0; u < 8; u++) v[u] = row[min(lane + 64 * u, n - 1)];   // clamped: no waits
#pragma unroll
      for (int u = 0; u < 8; u++) {
        const int j = lane + 64 * u;
        if (j < n) wrow[j] = (int32_t)mod_c((double)v[u], p, pinv);
      }
    }
    if (t == 0) *flag = 0;
    __syncthreads();
    for (int j0 = 0; j0 < n; j0 += PB) {
      const int pb = min(PB, n - j0);
      panel_body<PB, RPT, T>(W, ldw, n, j0, pb, p, pinv, piv, flag, linv, nullptr, n, sP);
      __syncthreads();                           // panel written back, swaps done, L11^{-1} stored
      const int r0 = j0 + pb, M = n - r0;
      if (M <= 0) break;
      // Loads below are unconditional, from indices clamped into range, and
      // the padding is selected when they are stored: a load under a
      // condition becomes a branch that waits for its own data.
      constexpr int NTL = (PB * PB + T - 1) / T;
      int32_t vt[NTL];
#pragma unroll
      for (int u = 0; u < NTL; u++) {
        const int e = u * T + t;
        vt[u] = linv[min(e / PB, pb - 1) * PB + min(e % PB, pb - 1)];
      }
#pragma unroll
      for (int u = 0; u < NTL; u++) {
        const int e = u * T + t, r = e / PB, c = e % PB;
        if (e < PB * PB) sT[r][c] = (r < pb && c < pb) ? (double)vt[u] : 0.0;
      }
      // the strip A12 = rows [j0, j0 + pb) x columns [r0, n), eight loads in
      // flight a thread; rows k >= pb and columns past M are zero
      const int M64 = (M + 63) / 64 * 64;
      for (int e0 = 0; e0 < PB * M64; e0 += 8 * T) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int e = e0 + u * T + t, k = e / M64, c = e % M64;
          v[u] = W[(int64_t)(j0 + min(k, pb - 1)) * ldw + r0 + min(c, M - 1)];
        }
#pragma unroll
        for (int u = 0; u < 8; u++) {
          const int e = e0 + u * T + t, k = e / M64, c = e % M64;
          if (e < PB * M64) sS[k * SW + c] = (k < pb && c < M) ? v[u] : 0;
        }
      }
      __syncthreads();
      // U12 = L11^{-1} A12 over the strip: 16-column blocks, block b of wave
      // w for b = w, w + 4, ...; a wave reads and rewrites only its own columns
      for (int b = wave; b < M64 / 16; b += 4) {
        v4d_q acc[PB / 16];
#pragma unroll
        for (int br = 0; br < PB / 16; br++) acc[br] = (v4d_q){0.0, 0.0, 0.0, 0.0};
        int steps = 0;
#pragma unroll
        for (int ks = 0; ks < PB; ks += 4) {
          const int kr = ks + (lane >> 4);
          const double bf = (double)sS[kr * SW + b * 16 + (lane & 15)];
#pragma unroll
          for (int br = 0; br < PB / 16; br++)
            acc[br] = __builtin_amdgcn_mfma_f64_16x16x4f64(sT[br * 16 + (lane & 15)][kr], bf,
                                                           acc[br], 0, 0, 0);
          if (++steps == kc4) {
            steps = 0;
#pragma unroll
            for (int br = 0; br < PB / 16; br++)
#pragma unroll
              for (int r = 0; r < 4; r++) acc[br][r] = mod_c(acc[br][r], p, pinv);
          }
        }
#pragma unroll
        for (int br = 0; br < PB / 16; br++)
#pragma unroll
          for (int r = 0; r < 4; r++)
            sS[(br * 16 + (lane >> 4) + 4 * r) * SW + b * 16 + (lane & 15)] =
                (int32_t)mod_c(acc[br][r], p, pinv);
      }
      __syncthreads();
      // A22 -= L21 U12 over the 64 x 64 tiles (row-major order); wave (wr, wc)
      // owns the 32 x 32 quarter as 2 x 2 MFMA blocks; the next tile's old
      // values are loaded while this one's products run
      const int nct = M64 / 64, ntile = nct * nct;
      int32_t vc[2][2][4], vn[2][2][4];
      auto load_c = [&](int idx, int32_t (&v)[2][2][4]) {
        const int rt = (idx / nct) * 64, ct = (idx % nct) * 64;
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
              const int gr = rt + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
              const int gc = ct + wc * 32 + j * 16 + (lane & 15);
              v[i][j][r] = W[(int64_t)(r0 + min(gr, M - 1)) * ldw + r0 + min(gc, M - 1)];
            }
      };
      load_c(0, vc);
      for (int idx = 0; idx < ntile; idx++) {
        if (idx + 1 < ntile) load_c(idx + 1, vn);
        const int rt = (idx / nct) * 64, ct = (idx % nct) * 64;
        v4d_q acc[2][2];
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int j = 0; j < 2; j++) acc[i][j] = (v4d_q){0.0, 0.0, 0.0, 0.0};
        int steps = 0;
#pragma unroll
        for (int ks = 0; ks < PB; ks += 4) {
          const int kr = ks + (lane >> 4);
          double af[2], bf[2];
#pragma unroll
          for (int i = 0; i < 2; i++) {
            const int pr = pb + rt + wr * 32 + i * 16 + (lane & 15);   // row of the panel
            af[i] = (pr < n - j0 && kr < pb) ? (double)sP[pr * SP + kr] : 0.0;
          }
#pragma unroll
          for (int j = 0; j < 2; j++) bf[j] = (double)sS[kr * SW + ct + wc * 32 + j * 16 + (lane & 15)];
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
              const int gr = rt + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
              const int gc = ct + wc * 32 + j * 16 + (lane & 15);
              if (gr < M && gc < M)
                W[(int64_t)(r0 + gr) * ldw + r0 + gc] =
                    (int32_t)mod_c((double)vc[i][j][r] - mod_c(acc[i][j][r], p, pinv), p, pinv);
            }
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
          for (int j = 0; j < 2; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) vc[i][j][r] = vn[i][j][r];
      }
      __syncthreads();                           // the trailing block is written
    }
    // K6: det mod p = (-1)^swaps prod u_jj
    double prod = 1.0;
    int swaps = 0;
    for (int j = t; j < n; j += T) {
      prod = mul_mod(prod, (double)W[(int64_t)j * ldw + j], p, pinv);
      swaps += piv[j] != j;
    }
    double* red = (double*)sS;
    red[t] = prod;
    const int odd = __syncthreads_count(swaps & 1) & 1;
    for (int s2 = T / 2; s2 > 0; s2 >>= 1) {
      if (t < s2) red[t] = mul_mod(red[t], red[t + s2], p, pinv);
      __syncthreads();
    }
    if (t == 0) {
      double d = red[0];
      if (odd) d = -d;
      if (*flag) d = 0.0;
      __hip_atomic_store(out + I.out_index, to_canonical(d, p), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
  }
}

// 0 for every counter of a queue (a kernel rather than a memset, so the reset
// can sit inside a captured graph).
__global__ void k_queue_reset(unsigned* next, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) next[i] = 0u;
}

int lu_queue_max_n(int variant) {
  return variant == LU_QUEUE_PB32 || variant == LU_QUEUE_PB16 || variant == LU_QUEUE_PB16X2 ? 512 : 0;
}

int64_t lu_queue_aux_stride() { return 512 + 4 + 32 * 32 + 60; }

int lu_queue_blocks_per_cu(int variant) { return variant == LU_QUEUE_PB16X2 ? 2 : 1; }

hipError_t launch_queue_reset(unsigned* next, int count, hipStream_t st) {
  k_queue_reset<<<(count + 255) / 256, 256, 0, st>>>(next, count);
  return hipGetLastError();
}

hipError_t launch_lu_queue(int variant, int grid, const LuItem* items, int nitems, unsigned* next,
                           int32_t* ws, int64_t ws_stride, int32_t* aux, uint32_t* out,
                           hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (grid <= 0) return hipErrorInvalidValue;
  const int64_t as = lu_queue_aux_stride();
  if (variant == LU_QUEUE_PB32)
    k_lu_queue<32, 2, 1><<<grid, 256, 0, st>>>(items, nitems, next, ws, ws_stride, aux, as, out);
  else if (variant == LU_QUEUE_PB16)
    k_lu_queue<16, 2, 1><<<grid, 256, 0, st>>>(items, nitems, next, ws, ws_stride, aux, as, out);
  else if (variant == LU_QUEUE_PB16X2)
    k_lu_queue<16, 2, 2><<<grid, 256, 0, st>>>(items, nitems, next, ws, ws_stride, aux, as, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace detk
