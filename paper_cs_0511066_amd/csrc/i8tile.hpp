// Three-limb int8 products on MFMA, shared by the LU's trailing update and
// the Hensel products of the lifting.
//
// A value r with -0x808080 <= r <= 0x7F7F7F is the sum of three signed
// bytes b_j 2^(8j): with u = r + 0x808080 (0 <= u < 2^24) and u_j the bytes
// of u, r = sum (u_j - 128) 2^(8j), and u_j - 128 is the byte u_j ^ 0x80
// read as a signed byte.  So the three limbs are bytes 0..2 of
// (r + 0x808080) ^ 0x808080.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace detk {

typedef int v4i_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t limb_word(int32_t r) {
  return (uint32_t)(r + 0x808080) ^ 0x808080u;
}

// K chunk of the tile product and the LDS row stride (80 B: 16-byte reads
// conflict-free).
constexpr int I8_TILE = 64, I8_K = 64, I8_LD = I8_K + 16;

// Limb planes: P[plane][row][k] (Rp x Kp bytes a plane, k contiguous, zero
// padded to multiples of 64).  One 256-thread workgroup accumulates the 64 x 64
// tile at (row0, col0) of A B^T over all Kp: A rows from PA, B rows (the
// columns of the product) from PB.  acc[s][i][j] = sum over a + b = s of
// A_a B_b for the 16 x 16 block (i, j) of wave (wr, wc) = (w >> 1, w & 1),
// 32 x 32 a wave; element r of lane l is row 4 (l / 16) + r, column l % 16 of
// the block.  Exact in int32 while 3 Kp 2^14 < 2^31.  The next chunk's loads
// are in flight during a chunk's products.
__device__ __forceinline__ void i8_tile_product(const int8_t* __restrict__ Az,
                                                const int8_t* __restrict__ Bz, int64_t planeA,
                                                int64_t planeB, int Kp, int row0, int col0,
                                                int8_t (*sA)[I8_TILE][I8_LD],
                                                int8_t (*sB)[I8_TILE][I8_LD],
                                                v4i_t (&acc)[5][2][2]) {
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  // 3 planes x 64 rows x 64 bytes per operand = 768 chunks of 16 B; 3 a thread
  v4i_t ga[3], gb[3];
  auto gload = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 3; u++) {
      const int e = t + u * 256;
      const int pl = e >> 8, rem = e & 255, r = rem >> 2, q = (rem & 3) * 16;
      ga[u] = *(const v4i_t*)(Az + pl * planeA + (int64_t)(row0 + r) * Kp + k0 + q);
      gb[u] = *(const v4i_t*)(Bz + pl * planeB + (int64_t)(col0 + r) * Kp + k0 + q);
    }
  };
#pragma unroll
  for (int s = 0; s < 5; s++)
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++) acc[s][i][j] = (v4i_t){0, 0, 0, 0};
  gload(0);
  for (int k0 = 0; k0 < Kp; k0 += I8_K) {
#pragma unroll
    for (int u = 0; u < 3; u++) {
      const int e = t + u * 256;
      const int pl = e >> 8, rem = e & 255, r = rem >> 2, q = (rem & 3) * 16;
      *(v4i_t*)(&sA[pl][r][q]) = ga[u];
      *(v4i_t*)(&sB[pl][r][q]) = gb[u];
    }
    __syncthreads();
    if (k0 + I8_K < Kp) gload(k0 + I8_K);
    v4i_t af[3][2], bf[3][2];
#pragma unroll
    for (int pl = 0; pl < 3; pl++) {
#pragma unroll
      for (int i = 0; i < 2; i++)
        af[pl][i] = *(const v4i_t*)(&sA[pl][wr * 32 + i * 16 + (lane & 15)][16 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < 2; j++)
        bf[pl][j] = *(const v4i_t*)(&sB[pl][wc * 32 + j * 16 + (lane & 15)][16 * (lane >> 4)]);
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++) {
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
          for (int b = 0; b < 3; b++)
            acc[a + b][i][j] =
                __builtin_amdgcn_mfma_i32_16x16x64_i8(af[a][i], bf[b][j], acc[a + b][i][j], 0, 0, 0);
      }
    __syncthreads();
  }
}

// Limb planes of 64 x 64 tiles of a matrix: the block of `rows` x K values
// v(r, k) (row-major) or, with `transpose`, of the K x rows block stored the
// other way (column j's K values become plane row j), read by `get`, written
// as P[3][Rp][Kp] (zero padding outside rows x K).  Tile (blockIdx.y,
// blockIdx.x) of output rows and k; 256 threads.  get(sr, sc) returns the
// source value at source row sr, column sc (indices in range).
template <class Get>
__device__ __forceinline__ void limb_split_tile(Get get, int rows, int K, int Kp, int64_t Rp,
                                                int transpose, int8_t* __restrict__ Pz,
                                                uint32_t (*sT)[65]) {
  const int t = threadIdx.x;
  const int ty = blockIdx.y * 64, tx = blockIdx.x * 64;   // tile: output rows ty.., k tx..
  // source tile: rows (ty.. for A, tx.. for B) x 64 columns; 16 values a thread
  const int sr0 = transpose ? tx : ty, sc0 = transpose ? ty : tx;
  const int srows = transpose ? K : rows, scols = transpose ? rows : K;
  int32_t x[16];
#pragma unroll
  for (int u = 0; u < 16; u++) {                // every load in flight before any use
    const int e = u * 256 + t, r = e >> 6, c = e & 63;
    x[u] = get(min(sr0 + r, srows - 1), min(sc0 + c, scols - 1));
  }
#pragma unroll
  for (int u = 0; u < 16; u++) {
    const int e = u * 256 + t, r = e >> 6, c = e & 63;
    sT[r][c] = limb_word((sr0 + r < srows && sc0 + c < scols) ? x[u] : 0);
  }
  __syncthreads();
  // output: 64 rows x 16 words of four k values, per plane; 4 words a thread
  const int64_t plane = Rp * (int64_t)Kp;
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const int e = u * 256 + t, orow = e >> 4, kq = (e & 15) * 4;
    uint32_t w[4];
#pragma unroll
    for (int q = 0; q < 4; q++) w[q] = transpose ? sT[kq + q][orow] : sT[orow][kq + q];
#pragma unroll
    for (int pl = 0; pl < 3; pl++) {
      // bytes pl of w0, w1 (and of w2, w3), then the two halves together
      const uint32_t sel = (uint32_t)pl | (uint32_t)(pl + 4) << 8 | 0x0c0c0000u;
      const uint32_t lo = __builtin_amdgcn_perm(w[1], w[0], sel);
      const uint32_t hi = __builtin_amdgcn_perm(w[3], w[2], sel);
      const uint32_t word = __builtin_amdgcn_perm(hi, lo, 0x05040100u);
      *(uint32_t*)(Pz + pl * plane + (int64_t)(ty + orow) * Kp + tx + kq) = word;
    }
  }
}

}  // namespace detk
