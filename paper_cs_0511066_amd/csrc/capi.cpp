// C-ABI of the library (include/det.h): contexts, the blocked LU driver,
// det_mod_primes, dixon_lift and det_introspective.  Every device step runs
// in the HIP kernels of lu_kernels.hip and dixon_kernels.hip; the host keeps
// prime sampling, Chinese remaindering with early termination, the p-adic to
// integer conversion, rational reconstruction and the final product.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <exception>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/det.h"
#include "../../include/det_host.h"
#include "bigint.hpp"
#include "host_numerics.hpp"
#include "kernels.hpp"
#include "ctx.hpp"

using dethost::BigInt;
using detk::Modulus;

namespace {

constexpr int NB_OUTER = 128;      // outer block (trailing-update depth K) of large batches
constexpr int TINV_LD = 128;       // leading dimension of the outer triangular inverses
constexpr int MAX_N = 4096;
// Batches below this size use single-level blocking (block = panel, so the
// panel's own L11^{-1} serves the triangular solve); larger batches use outer
// blocks of NB_OUTER columns so that the trailing update contracts over 128.
constexpr int TWO_LEVEL_MIN_ITEMS = 64;
// liftings side by side when det_opts.lift_primes is 0
constexpr int LIFT_PRIMES_AUTO = 4;

// Largest K such that K h^2 + h <= 2^53 with h = (pmax - 1)/2: FP64 sums of
// that many products of centred residues are exact.
int exact_chunk(uint32_t pmax) {
  const double h = (double)((pmax - 1) / 2);
  const double k = floor((9007199254740992.0 - h) / (h * h));
  return (int)std::min(k, 1e6);
}

Modulus modulus_of(uint32_t p) {
  Modulus m;
  m.p = (double)p;
  m.pinv = 1.0 / (double)p;
  return m;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Row stride of an LU workspace for rows of `w` entries: a multiple of 32
// entries plus 32, so that it is an odd multiple of 128 bytes (power-of-two
// strides put the rows of a tile on few memory channels).
int64_t lu_stride(int64_t w) { return round_up(w, 64) + 32; }

// Length of the zero-padded lifting vectors: the register-resident kernel
// reads 64 EPL entries (EPL = 4, 8, 16 for n <= 256, 512, 1024).
int64_t lift_pad(int64_t n) {
  if (n <= 256) return 256;
  if (n <= 512) return 512;
  if (n <= 1024) return 1024;
  return round_up(n, 64);
}

// ------------------------------------------------------------------ LU driver
struct LuJob {
  int n = 0;          // rows (and columns of A)
  int ncols = 0;      // n, or 2n for [A | I]
  int nitems = 0;     // batch items (one prime each)
  int64_t ldw = 0, slab = 0;
  bool int8 = false;  // trailing update on int8 limbs
  uint32_t pmax = 0;
  // columns [n, 2n) start as the identity ([A | I]): a step without row swaps
  // changes only the n columns [j0 + pb, n + j0 + pb), since row i of the
  // right half stays zero beyond column n + i until row i is a pivot row
  bool ident_right = false;
};

// Panels of one LU: first row, width, template width (ld of its inverses).
struct Panel {
  int j0, pb, pbw;
};

det_status gemm_update(det_ctx* c, LuWs& w, const LuJob& J, int64_t offC, int64_t offA,
                       int64_t offB, int M, int N, int K, int kc4, bool use_i8) {
  const int nit = J.nitems;
  const Modulus* mods = (const Modulus*)w.mods.p;
  int32_t* W = (int32_t*)w.W.p;
  if (M <= 0 || N <= 0 || K <= 0) return DET_OK;
  if (use_i8) {
    const int Kp = (int)((K + 63) / 64 * 64);
    const int64_t Mp = (M + 63) / 64 * 64, Np = (N + 63) / 64 * 64;
    const int64_t pslabA = 3 * Mp * Kp, pslabB = 3 * Np * Kp;
    TRY(ensure(c, w.limbA, (size_t)nit * pslabA, w.st));
    TRY(ensure(c, w.limbB, (size_t)nit * pslabB, w.st));
    // the timed interval covers the limb splits as well as the products
    ProfScope ps(c, DET_KERNEL_GEMM_I8,
                 (7.0 * (double)K * ((double)M + N) + 3.0 * Kp * (double)(Mp + Np) + 8.0 * M * N) * nit,
                 18.0 * M * N * K * nit, w.st);
    HIPCHK(detk::launch_split(W, J.slab, offA, J.ldw, M, K, Kp, Mp, 0, (int8_t*)w.limbA.p, pslabA,
                              nit, w.st));
    HIPCHK(detk::launch_split(W, J.slab, offB, J.ldw, N, K, Kp, Np, 1, (int8_t*)w.limbB.p, pslabB,
                              nit, w.st));
    HIPCHK(detk::launch_gemm_i8(W, J.slab, offC, J.ldw, M, N, (const int8_t*)w.limbA.p,
                                (const int8_t*)w.limbB.p, pslabA, pslabB, Mp, Np, Kp, mods, nit,
                                w.st));
  } else {
    ProfScope ps(c, DET_KERNEL_GEMM_F64,
                 4.0 * ((double)M * K + (double)K * N + 2.0 * M * N) * nit, 2.0 * M * N * K * nit,
                 w.st);
    HIPCHK(detk::launch_gemm_f64(W, J.slab, offC, offA, offB, J.ldw, M, N, K, mods, kc4, nit,
                                 w.st));
  }
  return DET_OK;
}

// ncols_sw > 0: the panel also applies its row swaps to the columns
// [j0 + pb, ncols_sw) right of it.
// rows_end > 0: the panel searches its pivots only in rows [j0, rows_end)
// (the diagonal block when the update forms L21 itself).
det_status panel_step(det_ctx* c, LuWs& w, const LuJob& J, const Panel& P, int32_t* uinv, int kc,
                      int ncols_sw = 0, int rows_end = 0) {
  const int nr = rows_end > 0 ? rows_end : J.n;
  const double m = nr - P.j0;
  ProfScope ps(c, DET_KERNEL_PANEL, 8.0 * m * P.pb * J.nitems, m * P.pb * P.pb * (double)J.nitems,
               w.st);
  HIPCHK(detk::launch_panel((int32_t*)w.W.p, J.ldw, J.slab, nr, P.j0, P.pb, P.pbw,
                            (const Modulus*)w.mods.p, (int32_t*)w.piv.p, J.n,
                            (int32_t*)w.flags.p, (int32_t*)w.linv.p, uinv, kc, J.nitems,
                            ncols_sw, w.st));
  return DET_OK;
}

// In-place X <- T X on rows [r0, r0+kb) x columns [c0, c0+N); with sw_pb > 0
// the panel's row swaps are applied to those columns first.
det_status trsm_step(det_ctx* c, LuWs& w, const LuJob& J, int r0, int kb, int c0, int N,
                     const int32_t* T, int ldt, int kc4, int sw_j0, int sw_pb) {
  if (kb <= 0 || N <= 0) return DET_OK;
  ProfScope ps(c, DET_KERNEL_TRSM, (8.0 * kb * N + 4.0 * kb * kb) * J.nitems,
               2.0 * kb * kb * N * J.nitems, w.st);
  HIPCHK(detk::launch_trsm_apply((int32_t*)w.W.p, J.slab, J.ldw, r0, kb, c0, N, T, ldt,
                                 (const Modulus*)w.mods.p, kc4, (const int32_t*)w.piv.p, J.n,
                                 sw_j0, sw_pb, J.nitems, w.st));
  return DET_OK;
}

// Blocked right-looking LU of every item (see lu_kernels.hip for the data
// layout).  W, piv, flags, mods of `w` must already hold residues and moduli.
// With keep_uinv (single item, single-level) the inverse of every panel's U11
// is kept in w.uinv for the back substitution; `panels` lists the panels.
// block_pivots (with keep_uinv, FP64): each panel looks for its pivots only in
// its diagonal block and the update forms L21 = A21 U11^{-1}; a column whose
// block has no non-zero entry raises the item's flag (the caller then runs
// the full pivot search).  Whenever no flag is raised the factors are those
// of an LU with the same row order, so the inverse and the determinant are
// unchanged: both are unique.
det_status lu_factor(det_ctx* c, LuWs& w, const LuJob& J, bool keep_uinv,
                     std::vector<Panel>* panels, bool block_pivots = false) {
  const int n = J.n, ncols = J.ncols, nit = J.nitems;
  const int64_t ldw = J.ldw;
  const int kc = exact_chunk(J.pmax);
  const int kc4 = std::max(1, kc / 4);
  const bool two_level = nit >= TWO_LEVEL_MIN_ITEMS;
  const int npan_max = n / 8 + 2;    // panels are at least 8 wide (the last may be narrower)
  // L11 inverses: two sets of nit x 32 x 32, used alternately by the steps
  // (a step's update may factor the next diagonal block while it reads its own)
  TRY(ensure(c, w.linv, (size_t)2 * nit * 32 * 32 * sizeof(int32_t), w.st));
  // U11 inverses: panel-major, one 32 x 32 slot per item (back_substitute
  // reads item 0's); with block pivots and no factors kept, two alternating sets
  if (keep_uinv)
    TRY(ensure(c, w.uinv, (size_t)npan_max * nit * 32 * 32 * sizeof(int32_t), w.st));
  else if (block_pivots)
    TRY(ensure(c, w.uinv, (size_t)2 * nit * 32 * 32 * sizeof(int32_t), w.st));
  const int32_t* linv = (const int32_t*)w.linv.p;
  if (panels) panels->clear();
  if (!two_level) {
    // FP64 trailing updates: the panel applies its swaps to the columns right
    // of it and one launch forms U12 and updates A22 (U12 kept, by the last
    // workgroup of each column tile to read A12, when the factors are needed:
    // per-step counters); int8: triangular apply, then the product
    const bool fused = !J.int8;
    const int cstride = (ncols + 63) / 64;
    unsigned* cnt = nullptr;
    if (fused && keep_uinv) {
      const size_t nc = (size_t)npan_max * nit * cstride;
      TRY(ensure(c, w.cnt, nc * sizeof(unsigned), w.st));
      HIPCHK(hipMemsetAsync(w.cnt.p, 0, nc * sizeof(unsigned), w.st));
      cnt = (unsigned*)w.cnt.p;
    }
    // U11^{-1} and L11^{-1} slots of step idx
    auto uinv_of = [&](int idx) -> int32_t* {
      if (keep_uinv) return (int32_t*)w.uinv.p + (size_t)idx * nit * 32 * 32;
      return block_pivots ? (int32_t*)w.uinv.p + (size_t)(idx & 1) * nit * 32 * 32 : nullptr;
    };
    auto linv_of = [&](int idx) { return (int32_t*)w.linv.p + (size_t)(idx & 1) * nit * 32 * 32; };
    bool diag_done = false;          // the previous step's update factored this diagonal block
    int idx = 0;
    for (int j0 = 0; j0 < n; idx++) {
      const int pbw = detk::panel_width_for(n - j0);
      const int pb = std::min(pbw, n - j0);
      const Panel P{j0, pb, pbw};
      if (idx >= npan_max) return fail(c, DET_E_INVALID, "panel count overflow");
      int32_t* uinv = uinv_of(idx);
      int32_t* lz = linv_of(idx);
      const bool bp = block_pivots && fused && uinv != nullptr;
      if (bp && pbw == 32) {
        if (!diag_done) {
          // the diagonal block alone (no row swaps)
          ProfScope ps(c, DET_KERNEL_PANEL, 8.0 * pb * pb * nit, (double)pb * pb * pb * nit, w.st);
          HIPCHK(detk::launch_diag_block((int32_t*)w.W.p, ldw, J.slab, j0, pb,
                                         (const Modulus*)w.mods.p, (int32_t*)w.piv.p, n,
                                         (int32_t*)w.flags.p, lz, uinv, nit, w.st));
        }
      } else {
        TRY(panel_step(c, w, J, P, uinv, kc, fused ? ncols : 0, bp ? j0 + pb : 0));
        // (the panel writes its L11^{-1} at the start of w.linv)
        lz = (int32_t*)w.linv.p;
      }
      diag_done = false;
      if (panels) panels->push_back(P);
      int right = ncols - (j0 + pb);
      if (J.ident_right && bp && pbw == 32) right = std::min(right, n);   // (no row swaps)
      if (fused) {
        const int M = n - (j0 + pb);
        // the next diagonal block inside this launch when it is 32 wide too
        const int next_pb = bp && pbw == 32 && M > 0 && detk::panel_width_for(M) == 32
                                ? std::min(32, M) : 0;
        ProfScope ps(c, DET_KERNEL_GEMM_F64,
                     4.0 * ((double)M * pb + (double)pb * right + 2.0 * (double)M * right) * nit,
                     2.0 * ((double)M + pb) * right * pb * nit, w.st);
        HIPCHK(detk::launch_lu_update((int32_t*)w.W.p, J.slab, ldw, j0, pb, M, right, lz, pbw,
                                      bp ? uinv : nullptr, (const Modulus*)w.mods.p, kc4,
                                      cnt ? cnt + (size_t)idx * nit * cstride : nullptr, cstride,
                                      nit, w.st, next_pb, next_pb ? linv_of(idx + 1) : nullptr,
                                      next_pb ? uinv_of(idx + 1) : nullptr, (int32_t*)w.piv.p, n,
                                      (int32_t*)w.flags.p));
        diag_done = next_pb > 0;
      } else {
        TRY(trsm_step(c, w, J, j0, pb, j0 + pb, right, linv, pbw, kc4, j0, pb));
        TRY(gemm_update(c, w, J, (int64_t)(j0 + pb) * ldw + j0 + pb,
                        (int64_t)(j0 + pb) * ldw + j0, (int64_t)j0 * ldw + j0 + pb,
                        n - (j0 + pb), right, pb, kc4, J.int8));
      }
      j0 += pb;
    }
    return DET_OK;
  }
  TRY(ensure(c, w.tinv, (size_t)nit * TINV_LD * TINV_LD * sizeof(int32_t), w.st));
  int32_t* tinv = (int32_t*)w.tinv.p;
  for (int k0 = 0; k0 < n; k0 += NB_OUTER) {
    const int kb = std::min(NB_OUTER, n - k0);
    for (int j0 = k0; j0 < k0 + kb;) {
      const int pbw = detk::panel_width_for(n - j0);
      const int pb = std::min(pbw, k0 + kb - j0);
      TRY(panel_step(c, w, J, Panel{j0, pb, pbw}, nullptr, kc));
      HIPCHK(detk::launch_swaps((int32_t*)w.W.p, ldw, J.slab, j0, pb, (const int32_t*)w.piv.p, n,
                                k0, j0, j0 + pb, ncols, nit, w.st));
      const int rest = k0 + kb - (j0 + pb);
      if (rest > 0) {
        TRY(trsm_step(c, w, J, j0, pb, j0 + pb, rest, linv, pbw, kc4, 0, 0));
        TRY(gemm_update(c, w, J, (int64_t)(j0 + pb) * ldw + j0 + pb,
                        (int64_t)(j0 + pb) * ldw + j0, (int64_t)j0 * ldw + j0 + pb, n - (j0 + pb),
                        rest, pb, kc4, false));
      }
      j0 += pb;
    }
    const int right = ncols - (k0 + kb);
    if (right <= 0) continue;
    {
      ProfScope ps(c, DET_KERNEL_TRI_INV, 8.0 * kb * kb * nit, (double)kb * kb * kb / 3.0 * nit,
                   w.st);
      HIPCHK(detk::launch_tri_inv((const int32_t*)w.W.p, ldw, J.slab, k0, kb,
                                  (const Modulus*)w.mods.p, tinv, TINV_LD, nit, w.st));
    }
    TRY(trsm_step(c, w, J, k0, kb, k0 + kb, right, tinv, TINV_LD, kc4, 0, 0));
    TRY(gemm_update(c, w, J, (int64_t)(k0 + kb) * ldw + k0 + kb, (int64_t)(k0 + kb) * ldw + k0,
                    (int64_t)k0 * ldw + k0 + kb, n - (k0 + kb), right, kb, kc4, J.int8));
  }
  return DET_OK;
}

// Back substitution U X = Y on [U | Y] (one item, after a single-level
// lu_factor with keep_uinv): X = U^{-1} Y = A^{-1} mod p, panel by panel
// from the bottom: X_blk = U11^{-1} Y_blk, then Y_above -= U_above,blk X_blk.
det_status back_substitute(det_ctx* c, LuWs& w, const LuJob& J, const std::vector<Panel>& panels,
                           int lu_items) {
  const int n = J.n;
  const int kc4 = std::max(1, exact_chunk(J.pmax) / 4);
  for (int idx = (int)panels.size() - 1; idx >= 0; idx--) {
    const Panel& P = panels[idx];
    const int32_t* uinv = (const int32_t*)w.uinv.p + (size_t)idx * lu_items * 32 * 32;
    TRY(trsm_step(c, w, J, P.j0, P.pb, n, n, uinv, P.pbw, kc4, 0, 0));
    if (P.j0 > 0)
      TRY(gemm_update(c, w, J, n, P.j0, (int64_t)P.j0 * J.ldw + n, P.j0, n, P.pb, kc4, false));
  }
  return DET_OK;
}

// A^{-1} = U^{-1} (L^{-1} P) from the factored [A | I] when every panel is 32
// wide, in a few launches for all items of the job: V = U^{-1} by recursive
// doubling over the diagonal blocks (for a pair of blocks of size b, V12 =
// -V1 U12 V2, batched over the pairs of a level and the items: the pairs lie
// a fixed stride 2b (ldw + 1) apart), then one product V (L^{-1} P) per
// item.  Regions of each item's slab (ldw >= 4n): [0, n) L\U, [n, 2n)
// L^{-1} P, [2n, 3n) V (cleared before the factorisation), [3n, 4n) scratch,
// then the inverse.
det_status inverse_from_lu(det_ctx* c, LuWs& w, const LuJob& J, int64_t* col_out) {
  const int n = J.n, nit = J.nitems;
  const int64_t ldw = J.ldw;
  const int kc4 = std::max(1, exact_chunk(J.pmax) / 4);
  const int64_t offV = 2 * (int64_t)n, offS = 3 * (int64_t)n;
  int32_t* W = (int32_t*)w.W.p;
  const Modulus* mods = (const Modulus*)w.mods.p;
  HIPCHK(detk::launch_place_diag(W, J.slab, ldw, offV, n, (const int32_t*)w.uinv.p, nit, w.st));
  for (int64_t b = 32; b < n; b *= 2) {
    const int64_t npairs = ((n + b - 1) / b) / 2;
    int64_t nfull = 0;
    while (nfull < npairs && (2 * nfull + 2) * b <= n) nfull++;
    // pairs i0 .. i0+cnt-1 of every item, right blocks of size r
    auto level = [&](int64_t i0, int64_t cnt, int64_t r) -> det_status {
      const int64_t rowL = 2 * i0 * b, rowR = rowL + b, stride = 2 * b * (ldw + 1);
      ProfScope ps(c, DET_KERNEL_GEMM_F64, 12.0 * b * (b + 2.0 * r) * cnt * nit,
                   2.0 * b * r * (r + b) * cnt * nit, w.st);
      HIPCHK(detk::launch_gemm_mod(W, stride, rowL * ldw + offS + rowR, rowL * ldw + rowR,
                                   rowR * ldw + offV + rowR, ldw, (int)b, (int)r, (int)r, mods, kc4,
                                   2, false, (int)cnt, w.st, nit, J.slab, true));   // S = U12 V2
      HIPCHK(detk::launch_gemm_mod(W, stride, rowL * ldw + offV + rowR, rowL * ldw + offV + rowL,
                                   rowL * ldw + offS + rowR, ldw, (int)b, (int)r, (int)b, mods, kc4,
                                   3, true, (int)cnt, w.st, nit, J.slab, true));    // V12 = -V1 S
      return DET_OK;
    };
    if (nfull > 0) TRY(level(0, nfull, b));
    if (npairs > nfull) TRY(level(nfull, 1, n - (2 * nfull + 1) * b));
  }
  {
    ProfScope ps(c, DET_KERNEL_GEMM_F64, 12.0 * (double)n * n * nit, (double)n * n * n * nit, w.st);
    HIPCHK(detk::launch_gemm_mod(W, J.slab, offS, offV, n, ldw, n, n, n, mods, kc4, 2, true, nit,
                                 w.st));
  }
  *col_out = offS;
  return DET_OK;
}

// Waits for `ev` (recorded already) by polling it: the host spins instead of
// sleeping in a blocking wait, which can leave it asleep for a few hundred
// microseconds after the device has finished.
det_status spin_event(det_ctx* c, hipEvent_t ev) {
  for (;;) {
    const hipError_t q = hipEventQuery(ev);
    if (q == hipSuccess) return DET_OK;
    if (q != hipErrorNotReady) return fail(c, DET_E_DEVICE, hipGetErrorString(q));
    __builtin_ia32_pause();
  }
}

// Waits for everything queued on st so far, by polling an event of its own.
det_status spin_stream(det_ctx* c, hipStream_t st) {
  hipEvent_t e = nullptr;
  HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  det_status r = DET_OK;
  if (hipEventRecord(e, st) != hipSuccess) r = fail(c, DET_E_DEVICE, "event record failed");
  else r = spin_event(c, e);
  (void)hipEventDestroy(e);
  return r;
}

// Validates A and returns a device pointer to it (uploading host memory into
// the context's A buffer) with its leading dimension.
det_status stage_matrix(det_ctx* c, const int64_t* A, int64_t n, int64_t lda,
                        const int64_t** dA, int64_t* dlda, bool* on_device) {
  *on_device = is_device_ptr(A);
  if (*on_device) {
    *dA = A;
    *dlda = lda;
    return DET_OK;
  }
  for (int64_t i = 0; i < n; i++)
    for (int64_t j = 0; j < n; j++) {
      const int64_t v = A[i * lda + j];
      if (v >= (1LL << 31) || v <= -(1LL << 31))
        return fail(c, DET_E_OVERFLOW, "matrix entry with |a_ij| >= 2^31");
    }
  TRY(ensure(c, c->Adev, (size_t)n * n * sizeof(int64_t)));
  HIPCHK(hipMemcpy2DAsync(c->Adev.p, n * sizeof(int64_t), A, lda * sizeof(int64_t),
                          n * sizeof(int64_t), n, hipMemcpyHostToDevice, c->st));
  *dA = (const int64_t*)c->Adev.p;
  *dlda = n;
  return DET_OK;
}

// Bounds of a staged matrix: on the host for host input, else by the norm
// kernels.  Also enforces |a_ij| < 2^31 for device input.
det_status matrix_bounds(det_ctx* c, const int64_t* A, int64_t lda, bool on_device,
                         const int64_t* dA, int64_t dlda, int64_t n, dethost::Bounds* b) {
  if (!on_device) {
    *b = dethost::bounds_host(A, n, lda);
    return DET_OK;
  }
  // column sums, row sums and row maxima in one buffer, read back with one
  // copy into pinned memory
  TRY(ensure(c, c->norms, ((size_t)3 * n + detk::norms_scratch((int)n)) * sizeof(double)));
  TRY(ensure_pin(c, c->hnorms, (size_t)3 * n * sizeof(double), c->st));
  double* dn = (double*)c->norms.p;
  HIPCHK(detk::launch_norms_wide(dA, dlda, (int)n, dn, dn + 2 * n, dn + 3 * n, c->st));
  const double* h = (const double*)c->hnorms.p;
  HIPCHK(hipMemcpyAsync((void*)h, dn, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  TRY(spin_stream(c, c->st));
  double amax = 0;
  for (int64_t i = 0; i < n; i++) amax = std::max(amax, h[2 * n + i]);
  if (amax >= 2147483648.0) return fail(c, DET_E_OVERFLOW, "matrix entry with |a_ij| >= 2^31");
  std::vector<double> cols(h, h + n), rows(h + n, h + 2 * n);
  *b = dethost::bounds_from_sums(cols, rows, amax);
  return DET_OK;
}

// Path of the trailing update for a batch: explicit choices are honoured;
// AUTO takes the int8 limbs when the batch is large enough for the deep
// (K = 128) contraction and every prime is below 2^23.
bool use_int8(det_path path, int64_t nitems, uint32_t pmax) {
  if (path == DET_PATH_INT8) return true;
  if (path == DET_PATH_FP64) return false;
  return nitems >= TWO_LEVEL_MIN_ITEMS && pmax < (1u << 23);
}

// Flags of a batch whose block-pivot check is left to the caller: primes
// [s0, s0 + count) of the call; flags (pinned host memory, valid after the
// workspace's stream is synchronized) non-zero where the block-pivot LU met a
// block column without a non-zero entry, so that the residue must be
// recomputed with the full pivot search.
struct Deferred {
  const int32_t* flags = nullptr;
  int64_t s0 = 0, count = 0;
};

// Modular determinants of a staged device matrix for a list of primes, in
// batches bounded by the workspace, on workspace w.  Single-level FP64
// batches first search pivots in each diagonal block (as the inverse does);
// a batch that meets a block column without a non-zero entry is computed
// again with the full search (allow_block false forces the full search).
// With `wait` false the last batch's residues are copied asynchronously into
// `out` (which must then be pinned memory), the caller synchronizes w.st and,
// when *deferred has a count, checks its flags and recomputes flagged primes.
det_status residues_core(det_ctx* c, LuWs& w, const int64_t* dA, int64_t dlda, int n,
                         const uint32_t* primes, int64_t np, uint32_t* out, det_path path,
                         bool wait = true, Deferred* deferred = nullptr, bool allow_block = true) {
  if (deferred) *deferred = Deferred();
  if (np == 0) return DET_OK;
  if (n == 0) {
    for (int64_t i = 0; i < np; i++) out[i] = 1 % primes[i];
    return DET_OK;
  }
  LuJob J;
  J.n = n;
  J.ncols = n;
  J.ldw = lu_stride(n);
  J.slab = J.ldw * n;
  const size_t per_item = (size_t)J.slab * 4 + 3 * (size_t)(2 * n) * NB_OUTER + TINV_LD * TINV_LD * 4;
  size_t cap_bytes = (size_t)8 << 30;                  // at most 8 GiB of slabs per batch
  if (c->budget) cap_bytes = std::min(cap_bytes, c->budget / 2);
  int64_t bmax = std::max<int64_t>(1, std::min<int64_t>(1024, (int64_t)(cap_bytes / per_item)));
  for (int64_t s0 = 0; s0 < np; s0 += bmax) {
    const int nit = (int)std::min<int64_t>(bmax, np - s0);
    J.nitems = nit;
    J.pmax = 0;
    HIPCHK(hipStreamSynchronize(w.st));             // the previous upload from hmods is done
    TRY(ensure_pin(c, w.hmods, (size_t)nit * sizeof(Modulus), w.st));
    TRY(ensure_pin(c, w.hflags, (size_t)nit * sizeof(int32_t), w.st));
    Modulus* hm = (Modulus*)w.hmods.p;
    for (int i = 0; i < nit; i++) {
      hm[i] = modulus_of(primes[s0 + i]);
      J.pmax = std::max(J.pmax, primes[s0 + i]);
    }
    J.int8 = use_int8(path, nit, J.pmax);
    const bool block = allow_block && c->block_pivots && !J.int8 && nit < TWO_LEVEL_MIN_ITEMS;
    TRY(ensure(c, w.W, (size_t)nit * J.slab * sizeof(int32_t), w.st));
    TRY(ensure(c, w.piv, (size_t)nit * n * sizeof(int32_t), w.st));
    TRY(ensure(c, w.flags, (size_t)nit * sizeof(int32_t), w.st));
    TRY(ensure(c, w.mods, (size_t)nit * sizeof(Modulus), w.st));
    TRY(ensure(c, w.res, (size_t)nit * sizeof(uint32_t), w.st));
    HIPCHK(hipMemcpyAsync(w.mods.p, hm, nit * sizeof(Modulus), hipMemcpyHostToDevice, w.st));
    HIPCHK(hipMemsetAsync(w.flags.p, 0, nit * sizeof(int32_t), w.st));
    {
      ProfScope ps(c, DET_KERNEL_RESIDUES, (double)n * n * (8.0 + 4.0 * nit), 0.0, w.st);
      HIPCHK(detk::launch_residues(dA, dlda, n, n, (int32_t*)w.W.p, J.ldw, J.slab,
                                   (const Modulus*)w.mods.p, nit, w.st));
    }
    TRY(lu_factor(c, w, J, false, nullptr, block));
    HIPCHK(detk::launch_det_finalize((const int32_t*)w.W.p, J.ldw, J.slab, n,
                                     (const int32_t*)w.piv.p, n, (const int32_t*)w.flags.p,
                                     (const Modulus*)w.mods.p, (uint32_t*)w.res.p, nit, w.st));
    HIPCHK(hipMemcpyAsync(out + s0, w.res.p, nit * sizeof(uint32_t), hipMemcpyDeviceToHost, w.st));
    if (block)
      HIPCHK(hipMemcpyAsync(w.hflags.p, w.flags.p, nit * sizeof(int32_t), hipMemcpyDeviceToHost,
                            w.st));
    const bool last = s0 + nit >= np;
    if (!wait && last) {
      if (block && deferred) {
        deferred->flags = (const int32_t*)w.hflags.p;
        deferred->s0 = s0;
        deferred->count = nit;
      } else if (block) {
        HIPCHK(hipStreamSynchronize(w.st));     // no caller check: check here
      } else {
        continue;
      }
      if (deferred) continue;
    } else {
      HIPCHK(hipStreamSynchronize(w.st));
    }
    if (block) {
      bool any = false;
      for (int i = 0; i < nit; i++) any |= ((const int32_t*)w.hflags.p)[i] != 0;
      if (any) {
        c->block_pivot_retries++;
        TRY(residues_core(c, w, dA, dlda, n, primes + s0, nit, out + s0, path, true, nullptr, false));
      }
    }
  }
  return DET_OK;
}

uint64_t inv_mod_2_64(uint64_t p) {
  uint64_t x = p;                         // correct to 3 bits for odd p
  for (int i = 0; i < 5; i++) x *= 2 - p * x;
  return x;
}

// A^{-1} mod p into c->Cu (canonical, n x n), from a staged device matrix,
// on workspace ws[0].  Returns DET_E_SINGULAR_MOD_P if p | det(A).
det_status ensure_pinned(det_ctx* c, size_t count);


// A^{-1} mod p_z into c->Cu + z n^2 (canonical, n x n) for np primes at once
// (np > 1 needs n <= 1024; the items of one batched LU of [A | I]), on
// workspace ws[0].  Returns DET_E_SINGULAR_MOD_P if some p_z divides det(A).
// With `deferred` (and the block pivot search on) only the block search runs
// and nothing waits for it: the np flags that say a block column had no
// non-zero entry are copied to the pinned words (*deferred)[0 .. np), valid
// once the caller has synchronised c->st; if one is set the caller discards
// what it computed from c->Cu and calls again without `deferred`.  With
// det_out (pinned, np words) det(A) mod p_z is read back from the same
// factorisation, with the flags, and det_done is recorded after both (a
// residue is valid when its flag is clear).
det_status inverse_mod_primes(det_ctx* c, const int64_t* dA, int64_t dlda, int n,
                              const uint32_t* ps, int np, const int32_t** deferred = nullptr,
                              uint32_t* det_out = nullptr, hipEvent_t det_done = nullptr) {
  LuWs& w = c->ws[0];
  // with every panel 32 wide the inverse is formed from the factors in a few
  // launches (inverse_from_lu, four n-wide regions), else by the blocked back
  // substitution (two)
  const bool fast = detk::panel_width_for(n) == 32;
  if (np < 1 || np > detk::LIFT_MAX_PRIMES || (np > 1 && !fast))
    return fail(c, DET_E_INVALID, "inverse: unsupported number of primes");
  LuJob J;
  J.n = n;
  J.ncols = 2 * n;
  J.ldw = lu_stride((fast ? 4 : 2) * (int64_t)n);
  J.slab = J.ldw * n;
  J.nitems = np;
  J.pmax = 0;
  for (int z = 0; z < np; z++) J.pmax = std::max(J.pmax, ps[z]);
  J.int8 = false;
  J.ident_right = true;
  TRY(ensure_pin(c, w.hmods, (size_t)np * sizeof(Modulus), w.st));
  TRY(ensure_pinned(c, 64));                       // c->hres[0..63]; a background CRA batch
  Modulus* hm = (Modulus*)w.hmods.p;               // writes from c->hres + 64
  for (int z = 0; z < np; z++) hm[z] = modulus_of(ps[z]);
  TRY(ensure(c, w.W, (size_t)np * J.slab * sizeof(int32_t), w.st));
  TRY(ensure(c, w.piv, (size_t)np * n * sizeof(int32_t), w.st));
  TRY(ensure(c, w.flags, (size_t)np * sizeof(int32_t), w.st));
  TRY(ensure(c, w.mods, (size_t)np * sizeof(Modulus), w.st));
  TRY(ensure(c, c->Cu, (size_t)np * n * n * sizeof(uint32_t)));
  HIPCHK(hipMemcpyAsync(w.mods.p, hm, (size_t)np * sizeof(Modulus), hipMemcpyHostToDevice, w.st));
  std::vector<Panel> panels;
  int32_t* flag = (int32_t*)c->hres;
  // first with pivots searched inside each diagonal block only (the panels
  // then take a few rows instead of all of them); if some block column has
  // no non-zero entry, again with the full pivot search, whose flag means
  // that p divides det(A)
  if (deferred) *deferred = nullptr;
  for (int attempt = 0; attempt < 2; attempt++) {
    const bool block_pivots = attempt == 0 && c->block_pivots;
    if (attempt == 1 && !c->block_pivots) break;
    HIPCHK(hipMemsetAsync(w.flags.p, 0, (size_t)np * sizeof(int32_t), w.st));
    // [A | I], and with the fast inverse V = columns [2n, 3n) (read by
    // inverse_from_lu) cleared by the same launch: the identity's columns
    // past 2n are zero
    HIPCHK(detk::launch_residues(dA, dlda, n, (fast ? 3 : 2) * n, (int32_t*)w.W.p, J.ldw, J.slab,
                                 (const Modulus*)w.mods.p, np, w.st));
    TRY(lu_factor(c, w, J, true, &panels, block_pivots));
    if (det_out) {
      // det(A) mod p_z from the same factorisation (U's diagonal and the
      // pivots of [A | I] are those of A), a free CRA residue per prime
      TRY(ensure(c, w.res, (size_t)np * sizeof(uint32_t), w.st));
      HIPCHK(detk::launch_det_finalize((const int32_t*)w.W.p, J.ldw, J.slab, n,
                                       (const int32_t*)w.piv.p, n, (const int32_t*)w.flags.p,
                                       (const Modulus*)w.mods.p, (uint32_t*)w.res.p, np, w.st));
      HIPCHK(hipMemcpyAsync(det_out, w.res.p, (size_t)np * sizeof(uint32_t),
                            hipMemcpyDeviceToHost, w.st));
    }
    HIPCHK(hipMemcpyAsync(flag, w.flags.p, (size_t)np * sizeof(int32_t), hipMemcpyDeviceToHost,
                          w.st));
    if (det_out && det_done) HIPCHK(hipEventRecord(det_done, w.st));
    if (block_pivots && deferred) {
      *deferred = flag;
      break;
    }
    HIPCHK(hipStreamSynchronize(w.st));
    bool any = false;
    for (int z = 0; z < np; z++) any |= flag[z] != 0;
    if (!any) break;
    if (!block_pivots) return fail(c, DET_E_SINGULAR_MOD_P, "p divides det(A)");
    c->block_pivot_retries++;
  }
  int64_t col = n;
  if (fast) TRY(inverse_from_lu(c, w, J, &col));
  else TRY(back_substitute(c, w, J, panels, 1));
  HIPCHK(detk::launch_extract_inverse((const int32_t*)w.W.p, J.slab, J.ldw, col, n,
                                      (const Modulus*)w.mods.p, (uint32_t*)c->Cu.p, np, w.st));
  return DET_OK;
}

// A^{-1} mod p into c->Cu (see inverse_mod_primes).
det_status inverse_mod_p(det_ctx* c, const int64_t* dA, int64_t dlda, int n, uint32_t p,
                         const int32_t** deferred = nullptr) {
  return inverse_mod_primes(c, dA, dlda, n, &p, 1, deferred);
}

// Layout of the pinned staging buffer c->hstage for a lifting of order n
// with k digits: r (int64, up to LIFT3_MAX_RHS right-hand sides), digit 0 of
// r, three balanced digits a record (four words, up to LIFT3_MAX_RHS records
// a row, for up to LIFT_MAX_PRIMES primes), digit 1 of r, the combination vector, then k combination sums read
// back.
struct Stage {
  size_t r, rp0, d3, rp1, cvec, comb, total;
};
Stage stage_layout(int64_t n, int64_t k) {
  Stage s;
  s.r = 0;
  s.rp0 = s.r + 8 * (size_t)n * detk::LIFT3_MAX_RHS;
  s.d3 = s.rp0 + 4 * (size_t)n;
  s.rp1 = s.d3 + 16 * (size_t)n * detk::LIFT3_MAX_RHS * detk::LIFT_MAX_PRIMES;
  s.cvec = s.rp1 + 4 * (size_t)n;
  s.comb = (s.cvec + 4 * (size_t)n + 63) & ~(size_t)63;
  s.total = s.comb + 8 * (size_t)k;
  return s;
}

// Called by a lifting once its preparation (Hensel planes, staging) is
// queued and before the lifting itself is launched; setting *skip ends the
// lifting there (nothing launched after the preparation).
typedef std::function<det_status(bool*)> PreLaunch;

// The FP64 three-digit lifting is exact for p < 2^25 and n ||A|| p < 2^53.
bool lift3_applies(int n, double amax, uint32_t p) {
  return p < (1u << 25) && (double)n * std::max(amax, 1.0) * (double)p < ldexp(1.0, 53);
}

// A as int32 (row-major, n x n) in c->Ai, for the Hensel planes and the
// lifting kernels (the entry bound |a_ij| < 2^31 is checked beforehand).
det_status pack_matrix(det_ctx* c, const int64_t* dA, int64_t dlda, int n) {
  TRY(ensure(c, c->Ai, (size_t)n * n * sizeof(int32_t)));
  HIPCHK(detk::launch_pack_i32(dA, dlda, n, (int32_t*)c->Ai.p, c->st));
  return DET_OK;
}

// Buffers of the three-digit lifting of order n for np primes, A packed into
// c->Ai, and the staging of the right-hand sides [h0, h0 + mm) of B (n x m,
// row-major): r_0 = b and its balanced digits mod p_z^3 (each centring
// carried into the next digit), one record of 25-bit fields under tag 0
// (step 0) per row, right-hand side and prime; xv filled with all-ones words
// (tag 127, not yet written by any step); the error word cleared.  Enqueued
// on c->st; the staging area is reused, so a second call must wait for the
// first one's copies.  The host computes the staging while the device still
// runs the inverse.
det_status lift3_stage(det_ctx* c, const int64_t* dA, int64_t dlda, int n, const int64_t* B,
                       int m, int h0, int mm, const uint32_t* ps, int np) {
  constexpr int MR = detk::LIFT3_MAX_RHS;
  const size_t nz = (size_t)np;
  if (np < 1 || np > detk::LIFT_MAX_PRIMES) return fail(c, DET_E_INVALID, "lifting: primes");
  if (h0 == 0) {
    TRY(pack_matrix(c, dA, dlda, n));
    TRY(ensure(c, c->C1, nz * n * n * sizeof(uint32_t)));
    TRY(ensure(c, c->C2, nz * n * n * sizeof(uint32_t)));
    TRY(ensure(c, c->Ed, nz * n * n * sizeof(double)));
    TRY(ensure(c, c->r, nz * n * MR * sizeof(int64_t)));
    TRY(ensure(c, c->rv, nz * n * MR * 4 * sizeof(uint32_t)));
    TRY(ensure(c, c->xv, nz * n * MR * 4 * sizeof(uint32_t)));
    TRY(ensure(c, c->sync, 64));
  }
  const Stage sl = stage_layout(n, 0);
  TRY(ensure_pin(c, c->hstage, sl.total, c->st));
  TRY(ensure_pin(c, c->hsmall, 64, c->st));
  char* hs = (char*)c->hstage.p;
  int64_t* hb = (int64_t*)(hs + sl.r);
  const size_t recs = (size_t)n * mm;
  for (int j = 0; j < n; j++)
    for (int hh = 0; hh < mm; hh++) hb[(size_t)j * mm + hh] = B[(size_t)j * m + h0 + hh];
  for (int z = 0; z < np; z++) {
    const int64_t pz = (int64_t)ps[z];
    uint32_t* d3 = (uint32_t*)(hs + sl.d3) + z * recs * 4;
    for (size_t e = 0; e < recs; e++) {
      int64_t v = hb[e];
      uint32_t* rec = d3 + e * 4;
      for (int q = 0; q < 3; q++) {
        int64_t md = v % pz;
        if (md < 0) md += pz;
        if (md > (pz - 1) / 2) md -= pz;
        rec[q] = (uint32_t)(int32_t)md & detk::LIFT3_DIGIT_MASK;
        v = (v - md) / pz;                             // exact
      }
      rec[3] = 0;
    }
    HIPCHK(hipMemcpyAsync((int64_t*)c->r.p + z * recs, hb, recs * sizeof(int64_t),
                          hipMemcpyHostToDevice, c->st));
  }
  HIPCHK(hipMemcpyAsync(c->rv.p, hs + sl.d3, nz * recs * 4 * sizeof(uint32_t),
                        hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemsetAsync(c->xv.p, 0xFF, nz * recs * 4 * sizeof(uint32_t), c->st));
  HIPCHK(hipMemsetAsync(c->sync.p, 0, 64, c->st));
  return DET_OK;
}

// The three-digit FP64 lifting (modulo p^3) of m right-hand sides B (n x m,
// row-major) for np primes side by side (Section 6: several p-adic liftings
// in parallel, each with fewer steps), from C0 = A^{-1} mod p_z in c->Cu + z
// n^2, on c->st: A packed into c->Ai, the Hensel planes of every prime in
// one batch, then one cooperative launch per LIFT3_MAX_RHS right-hand sides
// (they share the planes, the rows of A and every exchange; each prime has
// its own workgroups).  digits_dev: m x np x k x n, digit i of x_h modulo
// p_z at ((h np + z) k + i) n (may be null).  With after_own2 the launches
// first wait for own2.
// The Hensel planes on int8 MFMA when every operand fits three signed
// limbs (entries of A and centred residues within 0x7F7F7F), else FP64.
bool hensel_i8_applies(const det_ctx* c, double amax, const uint32_t* ps, int np) {
  if (!c->hensel_i8 || amax > (double)detk::LIMB3_MAX) return false;
  for (int z = 0; z < np; z++)
    if (ps[z] > 2u * (uint32_t)detk::LIMB3_MAX + 1u) return false;
  return true;
}

det_status lift3_multi(det_ctx* c, int grid3, const int64_t* dA, int64_t dlda, int n,
                       double amax, const int64_t* B, int m, const uint32_t* ps, int np, int64_t k,
                       uint32_t* digits_dev, bool after_own2, const int** err_pending = nullptr,
                       const PreLaunch* pre = nullptr) {
  const double nn = (double)n * n;
  if (np < 1 || np > detk::LIFT_MAX_PRIMES) return fail(c, DET_E_INVALID, "lifting: primes");
  const int mr = detk::lift3_max_rhs(n);
  // the first chunk's staging goes ahead of the Hensel products, so that the
  // lifting follows them (or the wait for own2) at once
  TRY(lift3_stage(c, dA, dlda, n, B, m, 0, std::min(mr, m), ps, np));
  int* err = (int*)((char*)c->sync.p + 32);
  int* herr = (int*)c->hsmall.p;
  if (hensel_i8_applies(c, amax, ps, np)) {
    TRY(ensure(c, c->Hp, detk::hensel_i8_scratch(n, np)));
    HIPCHK(detk::launch_hensel_i8((const int32_t*)c->Ai.p, (const uint32_t*)c->Cu.p,
                                  (double*)c->Ed.p, (uint32_t*)c->C1.p, (uint32_t*)c->C2.p, n, ps,
                                  np, (int8_t*)c->Hp.p, c->st));
  } else {
    HIPCHK(detk::launch_hensel_f64((const int32_t*)c->Ai.p, (const uint32_t*)c->Cu.p,
                                   (double*)c->Ed.p, (uint32_t*)c->C1.p, (uint32_t*)c->C2.p, n, ps,
                                   np, c->st));
  }
  if (pre) {
    bool skip = false;
    TRY((*pre)(&skip));
    if (skip) return DET_OK;
  }
  if (after_own2) {
    HIPCHK(hipEventRecord(c->ev, c->own2));
    HIPCHK(hipStreamWaitEvent(c->st, c->ev, 0));
  }
  for (int h0 = 0; h0 < m; h0 += mr) {
    const int mm = std::min(mr, m - h0);
    if (h0 > 0) {
      HIPCHK(hipStreamSynchronize(c->st));    // the staging of the last chunk is read
      TRY(lift3_stage(c, dA, dlda, n, B, m, h0, mm, ps, np));
    }
    {
      // algorithmic bytes per digit, right-hand side and prime: C and A as
      // the one-launch-per-phase form reads them (8 n^2) and four n-vectors
      ProfScope ps_(c, DET_KERNEL_LIFT, (8.0 * nn + 40.0 * n) * k * mm * np,
                    4.0 * nn * k * mm * np, c->st);
      HIPCHK(detk::launch_lift_resident3(
          grid3, (const uint32_t*)c->Cu.p, (const uint32_t*)c->C1.p, (const uint32_t*)c->C2.p,
          (const int32_t*)c->Ai.p, (int64_t*)c->r.p, (uint32_t*)c->rv.p, (uint32_t*)c->xv.p, n,
          mm, ps, np, k, digits_dev ? digits_dev + (size_t)h0 * np * k * n : nullptr,
          (int64_t)np * k * n, k * (int64_t)n, err, c->st));
    }
    HIPCHK(hipMemcpyAsync(herr, err, sizeof(int), hipMemcpyDeviceToHost, c->st));
    if (err_pending && h0 + mm >= m) {
      // the caller synchronises c->st later and then reads the word
      *err_pending = herr;
      break;
    }
    HIPCHK(hipStreamSynchronize(c->st));
    if (*herr) return fail(c, DET_E_DEVICE, "lifting: a wait for another workgroup's digits timed out");
  }
  return DET_OK;
}

// k Dixon steps from r_0 = b on c->st.  digits_dev: k x n output (may be null
// when only the combinations are wanted); comb_dev: k sums of cvec . x_i (may
// be null).
// The cooperative form needs all its workgroups resident at once, so when
// other work may be running on the context's second stream (`after_own2`),
// the launch first waits for that stream.  With `err_pending` the FP64
// three-digit form does not wait for the lifting: *err_pending is then the
// pinned word of its error flag, valid after the caller synchronises c->st
// (null when the form used has already checked it).
det_status lift(det_ctx* c, const int64_t* dA, int64_t dlda, int n, double amax, const int64_t* b,
                uint32_t p, int64_t k, uint32_t* digits_dev, const uint32_t* cvec_dev,
                uint64_t* comb_dev, bool after_own2 = false,
                const int** err_pending = nullptr, const PreLaunch* pre = nullptr) {
  if (err_pending) *err_pending = nullptr;
  const int grid3 = c->lift_mode == 0 && lift3_applies(n, amax, p) ? detk::lift3_grid(c->device, n) : 0;
  if (grid3 > 0) {    // lifting modulo p^3 in FP64: Hensel planes, then three digits a step
    uint32_t* dig = digits_dev;
    if (!dig && comb_dev) {
      TRY(ensure(c, c->digits, (size_t)k * n * sizeof(uint32_t)));
      dig = (uint32_t*)c->digits.p;
    }
    TRY(lift3_multi(c, grid3, dA, dlda, n, amax, b, 1, &p, 1, k, dig, after_own2, err_pending,
                    pre));
    if (comb_dev) HIPCHK(detk::launch_comb_digits(dig, k, n, cvec_dev, comb_dev, c->st));
    return DET_OK;
  }
  if (pre) {
    bool skip = false;
    TRY((*pre)(&skip));
    if (skip) return DET_OK;
  }
  TRY(pack_matrix(c, dA, dlda, n));
  // rp and x are padded with zeros to lift_pad(n) entries (the
  // register-resident kernel loads 64 EPL entries without bounds tests)
  const int64_t npad = lift_pad(n);
  TRY(ensure(c, c->r, (size_t)n * sizeof(int64_t)));
  TRY(ensure(c, c->rp, (size_t)npad * sizeof(uint32_t)));
  TRY(ensure(c, c->x, (size_t)npad * sizeof(uint32_t)));
  HIPCHK(hipMemsetAsync(c->rp.p, 0, npad * sizeof(uint32_t), c->st));
  HIPCHK(hipMemsetAsync(c->x.p, 0, npad * sizeof(uint32_t), c->st));
  const Stage sl = stage_layout(n, 0);
  TRY(ensure_pin(c, c->hstage, sl.total, c->st));
  TRY(ensure_pin(c, c->hsmall, 64, c->st));
  char* hs = (char*)c->hstage.p;
  int64_t* hb = (int64_t*)(hs + sl.r);
  uint32_t* rp0 = (uint32_t*)(hs + sl.rp0);
  for (int j = 0; j < n; j++) {
    hb[j] = b[j];
    int64_t m = b[j] % (int64_t)p;
    rp0[j] = (uint32_t)(m < 0 ? m + p : m);
  }
  HIPCHK(hipMemcpyAsync(c->r.p, hb, n * sizeof(int64_t), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(c->rp.p, rp0, n * sizeof(uint32_t), hipMemcpyHostToDevice, c->st));
  const uint64_t pinv64 = inv_mod_2_64(p);
  const double nn = (double)n * n;
  const int grid = c->lift_mode != 1 ? detk::lift_persistent_grid(c->device, n) : 0;
  if (grid > 0) {
    // lifting modulo p^2: Hensel step for the inverse, then two digits a step
    TRY(ensure(c, c->C1, (size_t)n * n * sizeof(uint32_t)));
    TRY(ensure(c, c->E, (size_t)n * n * sizeof(uint32_t)));
    TRY(ensure(c, c->rp1, (size_t)npad * sizeof(uint32_t)));
    TRY(ensure(c, c->x1, (size_t)npad * sizeof(uint32_t)));
    TRY(ensure(c, c->sync, 64));
    HIPCHK(hipMemsetAsync(c->rp1.p, 0, npad * sizeof(uint32_t), c->st));
    HIPCHK(hipMemsetAsync(c->x1.p, 0, npad * sizeof(uint32_t), c->st));
    HIPCHK(hipMemsetAsync(c->sync.p, 0, 64, c->st));
    // second base-p digit of b mod p^2
    uint32_t* rp1 = (uint32_t*)(hs + sl.rp1);
    for (int j = 0; j < n; j++) {
      const int64_t q = (b[j] - (int64_t)rp0[j]) / (int64_t)p;     // exact
      int64_t m = q % (int64_t)p;
      rp1[j] = (uint32_t)(m < 0 ? m + p : m);
    }
    HIPCHK(hipMemcpyAsync(c->rp1.p, rp1, n * sizeof(uint32_t), hipMemcpyHostToDevice, c->st));
    HIPCHK(detk::launch_hensel((const int32_t*)c->Ai.p, (const uint32_t*)c->Cu.p,
                               (uint32_t*)c->E.p, (uint32_t*)c->C1.p, n, p, c->st));
    if (after_own2) {
      HIPCHK(hipEventRecord(c->ev, c->own2));
      HIPCHK(hipStreamWaitEvent(c->st, c->ev, 0));
    }
    unsigned* bar = (unsigned*)c->sync.p;
    int* err = (int*)((char*)c->sync.p + 32);
    {
      // algorithmic bytes per digit: C and A as the one-launch-per-phase form
      // reads them (8 n^2) and four n-vectors
      ProfScope ps(c, DET_KERNEL_LIFT, (8.0 * nn + 40.0 * n) * k, 4.0 * nn * k, c->st);
      HIPCHK(detk::launch_lift_resident2(
          grid, (const uint32_t*)c->Cu.p, (const uint32_t*)c->C1.p, (const int32_t*)c->Ai.p,
          (int64_t*)c->r.p, (uint32_t*)c->rp.p, (uint32_t*)c->rp1.p, (uint32_t*)c->x.p,
          (uint32_t*)c->x1.p, n, p, pinv64, k, digits_dev, cvec_dev, comb_dev, bar, err, c->st));
    }
    int* herr = (int*)c->hsmall.p;
    HIPCHK(hipMemcpyAsync(herr, err, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (*herr) return fail(c, DET_E_DEVICE, "lifting grid barrier timed out");
    return DET_OK;
  }
  for (int64_t i = 0; i < k; i++) {
    uint32_t* xi = digits_dev ? digits_dev + i * n : (uint32_t*)c->x.p;
    {
      ProfScope ps(c, DET_KERNEL_LIFT_X, 4.0 * nn + 8.0 * n, 2.0 * nn, c->st);
      HIPCHK(detk::launch_lift_x((const uint32_t*)c->Cu.p, (const uint32_t*)c->rp.p, n, p, xi,
                                 c->st));
    }
    {
      ProfScope ps(c, DET_KERNEL_LIFT_R, 4.0 * nn + 24.0 * n, 2.0 * nn, c->st);
      HIPCHK(detk::launch_lift_r((const int32_t*)c->Ai.p, xi, (int64_t*)c->r.p,
                                 (uint32_t*)c->rp.p, n, p, pinv64, cvec_dev,
                                 comb_dev ? comb_dev + i : nullptr, c->st));
    }
  }
  HIPCHK(hipStreamSynchronize(c->st));     // rp0 lives on this frame
  return DET_OK;
}

det_status check_prime_list(det_ctx* c, const uint32_t* primes, int64_t np, uint32_t limit) {
  for (int64_t i = 0; i < np; i++) {
    const uint32_t q = primes[i];
    if (q >= limit || q < 3) return fail(c, DET_E_PRIME_RANGE, "prime outside the supported range");
    if (!dethost::is_prime_u32(q)) return fail(c, DET_E_NOT_PRIME, "modulus is not prime");
  }
  return DET_OK;
}

det_status ensure_pinned(det_ctx* c, size_t count) {
  if (c->hres_cap >= count) return DET_OK;
  if (c->hres) {
    HIPCHK(hipStreamSynchronize(c->own2));
    HIPCHK(hipHostFree(c->hres));
    c->hres = nullptr;
    c->hres_cap = 0;
  }
  const size_t cap = std::max<size_t>(count, 256);
  if (hipHostMalloc((void**)&c->hres, cap * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    c->hres = nullptr;
    return fail(c, DET_E_NOMEM, "hipHostMalloc failed");
  }
  c->hres_cap = cap;
  return DET_OK;
}

}  // namespace

// Entry points of the driver used by the batched and serving sources.
det_status drv_residues(det_ctx* c, LuWs& w, const int64_t* dA, int64_t dlda, int n,
                        const uint32_t* primes, int64_t np, uint32_t* out, det_path path) {
  return residues_core(c, w, dA, dlda, n, primes, np, out, path, true, nullptr, true);
}

det_status drv_check_primes(det_ctx* c, const uint32_t* primes, int64_t np, uint32_t limit) {
  return check_prime_list(c, primes, np, limit);
}

// ====================================================================== C ABI
extern "C" {

const char* det_status_str(det_status s) {
  switch (s) {
    case DET_OK: return "DET_OK";
    case DET_E_INVALID: return "DET_E_INVALID";
    case DET_E_NOT_PRIME: return "DET_E_NOT_PRIME";
    case DET_E_PRIME_RANGE: return "DET_E_PRIME_RANGE";
    case DET_E_SINGULAR_MOD_P: return "DET_E_SINGULAR_MOD_P";
    case DET_E_OVERFLOW: return "DET_E_OVERFLOW";
    case DET_E_NOMEM: return "DET_E_NOMEM";
    case DET_E_BUFFER_TOO_SMALL: return "DET_E_BUFFER_TOO_SMALL";
    case DET_E_DEVICE: return "DET_E_DEVICE";
  }
  return "DET_E_UNKNOWN";
}

const char* det_last_error(const det_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

det_status det_ctx_create(int device, size_t hbm_budget_bytes, det_ctx** out) {
  if (!out) return DET_E_INVALID;
  *out = nullptr;
  det_ctx* c = nullptr;
  try {
    c = new det_ctx();
  } catch (...) {
    return DET_E_NOMEM;
  }
  c->device = device;
  c->budget = hbm_budget_bytes;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count ||
      hipSetDevice(device) != hipSuccess ||
      hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&c->own2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_cra, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_det, hipEventDisableTiming) != hipSuccess ||
      hipEventCreate(&c->ev_t0) != hipSuccess || hipEventCreate(&c->ev_t1) != hipSuccess ||
      detk::configure_kernels() != hipSuccess) {
    (void)hipGetLastError();
    if (c->own) (void)hipStreamDestroy(c->own);
    if (c->own2) (void)hipStreamDestroy(c->own2);
    delete c;
    return DET_E_DEVICE;
  }
  c->st = c->own;
  c->ws[0].st = c->own;
  c->ws[1].st = c->own2;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    c->cus = prop.multiProcessorCount;
    snprintf(c->arch, sizeof(c->arch), "%s", prop.gcnArchName);
  }
  if (c->cus <= 0) c->cus = 1;
  const char* lm = getenv("DET_LIFT_MODE");     // "kernels": one launch per lifting phase
  if (lm && strcmp(lm, "kernels") == 0) c->lift_mode = 1;
  if (lm && strcmp(lm, "p2") == 0) c->lift_mode = 2;
  const char* bpv = getenv("DET_BLOCK_PIVOTS");   // "0": the inverse always searches whole columns
  c->block_pivots = !(bpv && strcmp(bpv, "0") == 0);
  const char* hm = getenv("DET_HENSEL");          // "f64": Hensel planes always on FP64 MFMA
  c->hensel_i8 = !(hm && strcmp(hm, "f64") == 0);
  *out = c;
  return DET_OK;
}

void det_ctx_destroy(det_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->st) (void)hipStreamSynchronize(c->st);
  if (c->own2) (void)hipStreamSynchronize(c->own2);
  std::vector<DevBuf*> all = {&c->Adev, &c->norms, &c->Cu, &c->Ai, &c->r, &c->rp,
                              &c->x, &c->digits, &c->comb, &c->cvec, &c->sync, &c->C1, &c->E,
                              &c->rp1, &c->x1, &c->C2, &c->Ed, &c->rv, &c->xv, &c->Hp, &c->q_items,
                              &c->q_next, &c->q_ws, &c->q_aux, &c->q_out, &c->q_mats};
  for (LuWs& w : c->ws)
    for (DevBuf* b : {&w.W, &w.piv, &w.flags, &w.mods, &w.linv, &w.uinv, &w.tinv, &w.limbA,
                      &w.limbB, &w.res, &w.cnt})
      all.push_back(b);
  for (DevBuf* b : all)
    if (b->p) (void)hipFree(b->p);
  if (c->hres) (void)hipHostFree(c->hres);
  for (PinBuf* pb : {&c->hstage, &c->hsmall, &c->hnorms, &c->hcomb, &c->ws[0].hmods, &c->ws[1].hmods,
                     &c->ws[0].hflags, &c->ws[1].hflags, &c->q_hitems, &c->q_hout})
    if (pb->p) (void)hipHostFree(pb->p);
  for (auto& pr : c->prof_pending) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->q_exec) (void)hipGraphExecDestroy(c->q_exec);
  if (c->ev) (void)hipEventDestroy(c->ev);
  if (c->ev_cra) (void)hipEventDestroy(c->ev_cra);
  if (c->ev_det) (void)hipEventDestroy(c->ev_det);
  if (c->ev_t0) (void)hipEventDestroy(c->ev_t0);
  if (c->ev_t1) (void)hipEventDestroy(c->ev_t1);
  if (c->own) (void)hipStreamDestroy(c->own);
  if (c->own2) (void)hipStreamDestroy(c->own2);
  delete c;
}

det_status det_ctx_set_stream(det_ctx* c, void* hip_stream) {
  if (!c) return DET_E_INVALID;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, DET_E_DEVICE, "hipSetDevice failed");
  HIPCHK(hipStreamSynchronize(c->st));
  c->st = hip_stream ? (hipStream_t)hip_stream : c->own;
  c->ws[0].st = c->st;
  return DET_OK;
}

void det_opts_default(det_opts* o) {
  if (!o) return;
  o->log2_inv_eps = 64.0;
  o->certify = 0;
  o->seed = 0x5DEECE66DULL;
  o->n_rhs = 1;
  o->prime_bits = 23;
  o->path = DET_PATH_AUTO;
  o->adaptive = 1;
  o->lift_primes = 0;
}

det_status det_profile_select(det_ctx* c, det_kernel kind) {
  if (!c || (int)kind < 0 || (int)kind > DET_KERNEL_LIFT) return DET_E_INVALID;
  c->prof_kind = (int)kind;
  return DET_OK;
}

det_status det_profile_read(det_ctx* c, int64_t* launches, double* total_ms, double* bytes,
                            double* ops) {
  if (!c) return DET_E_INVALID;
  HIPCHK(hipStreamSynchronize(c->st));
  HIPCHK(hipStreamSynchronize(c->own2));
  std::lock_guard<std::mutex> lk(c->mu);
  double ms = 0;
  for (auto& pr : c->prof_pending) {
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, pr.first, pr.second));
    ms += t;
    c->ev_pool.push_back(pr.first);
    c->ev_pool.push_back(pr.second);
  }
  c->prof_pending.clear();
  if (launches) *launches = c->prof_launches;
  if (total_ms) *total_ms = ms;
  if (bytes) *bytes = c->prof_bytes;
  if (ops) *ops = c->prof_ops;
  c->prof_launches = 0;
  c->prof_bytes = c->prof_ops = 0;
  return DET_OK;
}

det_status det_mod_primes(det_ctx* c, const int64_t* A, int64_t n, int64_t lda,
                          const uint32_t* primes, int64_t nprimes, uint32_t* residues,
                          det_path path) {
  if (!c) return DET_E_INVALID;
  try {
    if (n < 0 || nprimes < 0 || (n > 0 && (!A || lda < n)) || (nprimes > 0 && (!primes || !residues)))
      return fail(c, DET_E_INVALID, "invalid argument");
    if (n > MAX_N) return fail(c, DET_E_INVALID, "n exceeds 4096");
    if (path != DET_PATH_AUTO && path != DET_PATH_FP64 && path != DET_PATH_INT8)
      return fail(c, DET_E_INVALID, "unknown path");
    uint32_t pmax = 0;
    for (int64_t i = 0; i < nprimes; i++) pmax = std::max(pmax, primes[i]);
    const bool limb_range = path == DET_PATH_INT8;
    TRY(check_prime_list(c, primes, nprimes, limb_range ? (1u << 23) : (1u << 26)));
    if (n == 0 || nprimes == 0) {
      for (int64_t i = 0; i < nprimes; i++) residues[i] = 1 % primes[i];
      return DET_OK;
    }
    HIPCHK(hipSetDevice(c->device));
    const int64_t* dA;
    int64_t dlda;
    bool on_dev;
    TRY(stage_matrix(c, A, n, lda, &dA, &dlda, &on_dev));
    if (on_dev) {
      dethost::Bounds b;
      TRY(matrix_bounds(c, A, lda, true, dA, dlda, n, &b));
    }
    return residues_core(c, c->ws[0], dA, dlda, (int)n, primes, nprimes, residues, path);
  } catch (const std::exception& e) {
    return fail(c, DET_E_NOMEM, e.what());
  } catch (...) {
    return fail(c, DET_E_INVALID, "unexpected error");
  }
}

det_status dixon_lift(det_ctx* c, const int64_t* A, int64_t n, int64_t lda, const int64_t* b,
                      uint32_t p, int64_t k, uint32_t* digits) {
  if (!c) return DET_E_INVALID;
  try {
    if (n < 0 || k < 0 || (n > 0 && (!A || lda < n || !b)) || (n > 0 && k > 0 && !digits))
      return fail(c, DET_E_INVALID, "invalid argument");
    if (n > MAX_N) return fail(c, DET_E_INVALID, "n exceeds 4096");
    if (p <= 256 || p >= (1u << 26)) return fail(c, DET_E_PRIME_RANGE, "p must lie in (2^8, 2^26)");
    if (!dethost::is_prime_u32(p)) return fail(c, DET_E_NOT_PRIME, "p is not prime");
    if (n == 0 || k == 0) return DET_OK;
    const double blim = ldexp(1.0, 62) / (double)(n + 1);
    for (int64_t j = 0; j < n; j++)
      if (fabs((double)b[j]) >= blim) return fail(c, DET_E_OVERFLOW, "|b_j| too large");
    HIPCHK(hipSetDevice(c->device));
    const int64_t* dA;
    int64_t dlda;
    bool on_dev;
    TRY(stage_matrix(c, A, n, lda, &dA, &dlda, &on_dev));
    dethost::Bounds bd;
    TRY(matrix_bounds(c, A, lda, on_dev, dA, dlda, n, &bd));
    if ((double)n * bd.amax * (double)p >= ldexp(1.0, 62))
      return fail(c, DET_E_OVERFLOW, "n ||A|| p >= 2^62");
    TRY(inverse_mod_p(c, dA, dlda, (int)n, p));
    TRY(ensure(c, c->digits, (size_t)k * n * sizeof(uint32_t)));
    TRY(lift(c, dA, dlda, (int)n, bd.amax, b, p, k, (uint32_t*)c->digits.p, nullptr, nullptr));
    HIPCHK(hipMemcpyAsync(digits, c->digits.p, (size_t)k * n * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return DET_OK;
  } catch (const std::exception& e) {
    return fail(c, DET_E_NOMEM, e.what());
  } catch (...) {
    return fail(c, DET_E_INVALID, "unexpected error");
  }
}

det_status dixon_lift_primes(det_ctx* c, const int64_t* A, int64_t n, int64_t lda,
                             const int64_t* b, const uint32_t* primes, int64_t np, int64_t k,
                             uint32_t* digits) {
  if (!c) return DET_E_INVALID;
  try {
    if (n < 0 || k < 0 || np < 1 || np > detk::LIFT_MAX_PRIMES || !primes ||
        (n > 0 && (!A || lda < n || !b)) || (n > 0 && k > 0 && !digits))
      return fail(c, DET_E_INVALID, "invalid argument");
    if (n > MAX_N) return fail(c, DET_E_INVALID, "n exceeds 4096");
    for (int64_t z = 0; z < np; z++) {
      if (primes[z] <= 256 || primes[z] >= (1u << 26))
        return fail(c, DET_E_PRIME_RANGE, "p must lie in (2^8, 2^26)");
      if (!dethost::is_prime_u32(primes[z])) return fail(c, DET_E_NOT_PRIME, "p is not prime");
      for (int64_t y = 0; y < z; y++)
        if (primes[y] == primes[z]) return fail(c, DET_E_INVALID, "primes not distinct");
    }
    if (n == 0 || k == 0) return DET_OK;
    const double blim = ldexp(1.0, 62) / (double)(n + 1);
    for (int64_t j = 0; j < n; j++)
      if (fabs((double)b[j]) >= blim) return fail(c, DET_E_OVERFLOW, "|b_j| too large");
    HIPCHK(hipSetDevice(c->device));
    const int64_t* dA;
    int64_t dlda;
    bool on_dev;
    TRY(stage_matrix(c, A, n, lda, &dA, &dlda, &on_dev));
    dethost::Bounds bd;
    TRY(matrix_bounds(c, A, lda, on_dev, dA, dlda, n, &bd));
    uint32_t pmax = 0;
    bool three = c->lift_mode == 0;
    for (int64_t z = 0; z < np; z++) {
      pmax = std::max(pmax, primes[z]);
      three &= lift3_applies((int)n, bd.amax, primes[z]);
    }
    if ((double)n * bd.amax * (double)pmax >= ldexp(1.0, 62))
      return fail(c, DET_E_OVERFLOW, "n ||A|| p >= 2^62");
    const int grid3 = three ? detk::lift3_grid(c->device, (int)n) : 0;
    TRY(ensure(c, c->digits, (size_t)np * k * n * sizeof(uint32_t)));
    uint32_t* dig = (uint32_t*)c->digits.p;
    if (grid3 > 0 && np <= detk::lift3_max_primes(c->device, (int)n)) {
      // one batched inverse and one launch for every prime
      TRY(inverse_mod_primes(c, dA, dlda, (int)n, primes, (int)np));
      TRY(lift3_multi(c, grid3, dA, dlda, (int)n, bd.amax, b, 1, primes, (int)np, k, dig, false));
    } else {
      for (int64_t z = 0; z < np; z++) {
        TRY(inverse_mod_p(c, dA, dlda, (int)n, primes[z]));
        TRY(lift(c, dA, dlda, (int)n, bd.amax, b, primes[z], k, dig + (size_t)z * k * n, nullptr,
                 nullptr));
      }
    }
    HIPCHK(hipMemcpyAsync(digits, dig, (size_t)np * k * n * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return DET_OK;
  } catch (const std::exception& e) {
    return fail(c, DET_E_NOMEM, e.what());
  } catch (...) {
    return fail(c, DET_E_INVALID, "unexpected error");
  }
}

det_status dixon_lift_multi(det_ctx* c, const int64_t* A, int64_t n, int64_t lda,
                            const int64_t* B, int64_t m, uint32_t p, int64_t k, uint32_t* digits) {
  if (!c) return DET_E_INVALID;
  try {
    if (n < 0 || k < 0 || m < 0 || (n > 0 && (!A || lda < n)) || (n > 0 && m > 0 && !B) ||
        (n > 0 && k > 0 && m > 0 && !digits))
      return fail(c, DET_E_INVALID, "invalid argument");
    if (n > MAX_N) return fail(c, DET_E_INVALID, "n exceeds 4096");
    if (m > (1 << 20)) return fail(c, DET_E_INVALID, "m too large");
    if (p <= 256 || p >= (1u << 26)) return fail(c, DET_E_PRIME_RANGE, "p must lie in (2^8, 2^26)");
    if (!dethost::is_prime_u32(p)) return fail(c, DET_E_NOT_PRIME, "p is not prime");
    if (n == 0 || k == 0 || m == 0) return DET_OK;
    const double blim = ldexp(1.0, 62) / (double)(n + 1);
    for (int64_t e = 0; e < n * m; e++)
      if (fabs((double)B[e]) >= blim) return fail(c, DET_E_OVERFLOW, "|B_jh| too large");
    HIPCHK(hipSetDevice(c->device));
    const int64_t* dA;
    int64_t dlda;
    bool on_dev;
    TRY(stage_matrix(c, A, n, lda, &dA, &dlda, &on_dev));
    dethost::Bounds bd;
    TRY(matrix_bounds(c, A, lda, on_dev, dA, dlda, n, &bd));
    if ((double)n * bd.amax * (double)p >= ldexp(1.0, 62))
      return fail(c, DET_E_OVERFLOW, "n ||A|| p >= 2^62");
    TRY(inverse_mod_p(c, dA, dlda, (int)n, p));
    TRY(ensure(c, c->digits, (size_t)m * k * n * sizeof(uint32_t)));
    uint32_t* dig = (uint32_t*)c->digits.p;
    const int grid3 =
        c->lift_mode == 0 && lift3_applies((int)n, bd.amax, p) ? detk::lift3_grid(c->device, (int)n) : 0;
    if (grid3 > 0) {
      TRY(lift3_multi(c, grid3, dA, dlda, (int)n, bd.amax, B, (int)m, &p, 1, k, dig, false));
    } else {
      std::vector<int64_t> bh(n);
      for (int64_t h = 0; h < m; h++) {
        for (int64_t j = 0; j < n; j++) bh[j] = B[j * m + h];
        TRY(lift(c, dA, dlda, (int)n, bd.amax, bh.data(), p, k, dig + (size_t)h * k * n,
                 nullptr, nullptr));
      }
    }
    HIPCHK(hipMemcpyAsync(digits, dig, (size_t)m * k * n * sizeof(uint32_t), hipMemcpyDeviceToHost,
                          c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return DET_OK;
  } catch (const std::exception& e) {
    return fail(c, DET_E_NOMEM, e.what());
  } catch (...) {
    return fail(c, DET_E_INVALID, "unexpected error");
  }
}

det_status det_introspective(det_ctx* c, const int64_t* A, int64_t n, int64_t lda,
                             const det_opts* opts_in, int* sign, uint32_t* mag, int64_t limb_cap,
                             int64_t* limb_count, det_report* report) {
  if (!c) return DET_E_INVALID;
  try {
    if (n < 0 || !sign || !limb_count || (n > 0 && (!A || lda < n)) || limb_cap < 0 ||
        (limb_cap > 0 && !mag))
      return fail(c, DET_E_INVALID, "invalid argument");
    if (n > MAX_N) return fail(c, DET_E_INVALID, "n exceeds 4096");
    det_opts o;
    det_opts_default(&o);
    if (opts_in) o = *opts_in;
    if (o.n_rhs < 1) o.n_rhs = 1;
    if (!(o.log2_inv_eps > 0)) o.log2_inv_eps = 64.0;
    if (o.path != DET_PATH_AUTO && o.path != DET_PATH_FP64 && o.path != DET_PATH_INT8)
      return fail(c, DET_E_INVALID, "unknown path");
    if (o.prime_bits < 12 || o.prime_bits > (o.path == DET_PATH_INT8 ? 23 : 26))
      return fail(c, DET_E_PRIME_RANGE, "prime_bits out of range");
    det_report rep;
    memset(&rep, 0, sizeof(rep));
    auto emit = [&](const BigInt& v) -> det_status {
      std::vector<uint32_t> l = v.limbs32();
      *sign = v.sign;
      *limb_count = (int64_t)l.size();
      if ((int64_t)l.size() > limb_cap) return fail(c, DET_E_BUFFER_TOO_SMALL, "limb_cap too small");
      if (!l.empty()) memcpy(mag, l.data(), l.size() * sizeof(uint32_t));
      return DET_OK;
    };
    if (n == 0) {
      if (report) *report = rep;
      return emit(BigInt::from_i64(1));
    }
    HIPCHK(hipSetDevice(c->device));
    const int64_t* dA;
    int64_t dlda;
    bool on_dev;
    TRY(stage_matrix(c, A, n, lda, &dA, &dlda, &on_dev));
    dethost::Bounds bd;
    TRY(matrix_bounds(c, A, lda, on_dev, dA, dlda, n, &bd));
    rep.hadamard_bits = (int64_t)ceil(bd.log2_h);
    uint64_t rng = o.seed;
    double t_host = 0;
    const int bits = o.prime_bits;
    const double log2_l = (double)(bits - 1);
    dethost::PrimeSampler samp(dethost::splitmix64(rng), bits);

    const double tl0 = now_ms();
    // 25-bit primes when the FP64 three-digit lifting applies, else the
    // largest below 2^26 with n ||A|| p < 2^62 (64-bit integer lifting)
    const bool three = c->lift_mode == 0 && lift3_applies((int)n, bd.amax, (1u << 25) - 1) &&
                       detk::lift3_grid(c->device, (int)n) > 0;
    int dixon_bits = three ? 25 : 26;
    // 24-bit primes (below 2 * 0x7F7F7F + 1) when the Hensel planes can then
    // come from int8 limbs: 4% more digits, against products several times
    // faster
    uint32_t dixon_cap = UINT32_MAX;
    if (three && c->hensel_i8 && bd.amax <= (double)detk::LIMB3_MAX) {
      dixon_bits = 24;
      dixon_cap = 2u * (uint32_t)detk::LIMB3_MAX + 1u;
    }
    while (dixon_bits > 12 && (double)n * bd.amax * ldexp(1.0, dixon_bits) >= ldexp(1.0, 62))
      dixon_bits--;
    const int64_t beta = std::max<int64_t>(2, (int64_t)ceil(bd.log2_h));
    const int i_max = std::min(std::max(o.n_rhs, 1), 8);
    bool batch1_taken = false;
    dethost::PrimeSampler dsamp(dethost::splitmix64(rng), dixon_bits);
    // Pass 0 takes the inverse with the block pivot search and does not wait
    // for its flag: the flag is read with the first CRA batch, before the
    // first lifting is launched, and if a block column had no non-zero entry
    // that lifting is not launched and pass 1 starts over with the full
    // search (and fresh primes).
    // Liftings side by side (Section 6: several p-adic liftings in parallel,
    // each with fewer steps, combined by Chinese remaindering): np primes,
    // each lifted to k digits with prod p_z^k above the bound, when the
    // three-digit form applies and np of its grids fit on the device.
    const int grid3 = three ? detk::lift3_grid(c->device, (int)n) : 0;
    int np = 1;
    if (grid3 > 0) {
      const int cap = detk::lift3_max_primes(c->device, (int)n);
      np = o.lift_primes > 0 ? std::min(o.lift_primes, cap) : std::min(cap, LIFT_PRIMES_AUTO);
      np = std::max(1, np);
    }
    rep.lift_primes = np;
    // The first lifting waits for both the first inverse (with its Hensel
    // step) and the first CRA batch, which take about as long as each other:
    // the batch's thread starts first, then the inverse is enqueued beside it
    // (the pinned read-back words both use are sized for the batch first, and
    // A is marked ready for the batch's stream).
    const double logl_H0 = std::max(1.0, bd.log2_h / log2_l);
    const int64_t k0 = dethost::et_run_length(o.log2_inv_eps, dethost::prime_set_size(bits), logl_H0);
    // (two more primes than the run: a determinant of up to two primes' worth
    // of bits ends the CRA within the batch; the inverse's LU adds residues
    // modulo the np lifting primes, so the batch is np primes shorter)
    const bool solving = bd.log2_h > 0 && dixon_bits > 12;
    const int64_t batch1 =
        k0 > 0 ? std::min<int64_t>(std::max<int64_t>(k0 + 2 - (solving ? np : 0), 4), 64) : 16;
    TRY(ensure_pinned(c, (size_t)batch1 + 64));
    HIPCHK(hipEventRecord(c->ev_cra, c->st));          // A (and its bounds) are ready on st
    auto draw_dixon = [&](uint32_t* dps) {
      for (int z = 0; z < np; z++) {
        bool fresh;
        do {
          dps[z] = dsamp.next();
          fresh = dps[z] <= dixon_cap;
          for (int y = 0; y < z; y++) fresh &= dps[y] != dps[z];
        } while (!fresh);
      }
    };
    std::vector<uint32_t> ps1(batch1);
    for (auto& q : ps1) q = samp.next();
    uint32_t* hres1 = c->hres + 64;                  // (c->hres[0..63]: the inverse's read-backs)
    // ---------------- CRA batch 1 on the second stream (Section 4: the
    // modular determinants run in the background while the systems are
    // solved).  Its size covers the run length of Lemma 2.1(iv) for the
    // bound H itself; once s_n is known, fewer may be needed.
    const double tc0 = now_ms();
    HIPCHK(hipStreamWaitEvent(c->own2, c->ev_cra, 0));
    // A second host thread enqueues the batch (some seventy launches) while
    // this one enqueues the inverse.  It uses only ws[1], own2 and hres1
    // (the inverse's read-backs are c->hres[0..63], already allocated); it is
    // joined before anything waits for own2.
    det_status cra_st = DET_OK;
    Deferred cra_def;
    std::thread cra_thread;
    struct Joiner {
      std::thread& t;
      std::function<void()> start;
      bool started = false;
      void run() {
        if (!started) {
          started = true;
          t = std::thread(start);
        }
      }
      void join() {
        run();
        if (t.joinable()) t.join();
      }
      ~Joiner() {
        if (t.joinable()) t.join();
      }
    } cra_join{cra_thread, [&] {
      try {
        (void)hipSetDevice(c->device);
        (void)hipEventRecord(c->ev_t0, c->own2);
        cra_st = residues_core(c, c->ws[1], dA, dlda, (int)n, ps1.data(), batch1, hres1, o.path,
                               false, &cra_def);
        (void)hipEventRecord(c->ev_t1, c->own2);
      } catch (...) {
        cra_st = DET_E_NOMEM;
      }
    }};
    cra_join.run();

    uint32_t dps0[detk::LIFT_MAX_PRIMES] = {0, 0, 0, 0};
    det_status st0 = DET_E_SINGULAR_MOD_P;
    const int32_t* inv_flag0 = nullptr;
    uint32_t* hdet0 = c->hres + 32;                  // det(A) mod the lifting primes
    if (solving) {
      draw_dixon(dps0);
      st0 = inverse_mod_primes(c, dA, dlda, (int)n, dps0, np, &inv_flag0, hdet0, c->ev_det);
    }

    // ---------------- The CRA loop on det(A)/K (Alg. 2.1 on the quotient,
    // Section 4): every residue computed so far is kept (d_i = det mod p_i)
    // and re-used whenever K grows (d_i K^{-1} mod p_i; primes dividing K are
    // skipped); new batches of primes run on ws[0] until early termination
    // (run length of Lemma 2.1(iv) for the bound H/K), the deterministic
    // bound prod p >= 2H/K, or, with a time budget, until the budget is spent.
    BigInt K = BigInt::from_i64(1);
    std::vector<uint32_t> cra_p, cra_r;             // primes and residues, in draw order
    dethost::CrtState crt;
    bool done = false;
    double t_lu_ms = 0, lu_primes = 0;              // device time per modular determinant
    auto restart_crt = [&]() {
      crt = dethost::CrtState();
      done = false;
    };
    auto feed = [&](size_t from) {                  // Garner steps for primes [from, end)
      const double log2_HK = std::max(0.0, bd.log2_h - (double)(K.bit_length() - 1));
      const double logl_H = std::max(1.0, log2_HK / log2_l);
      int64_t kET = dethost::et_run_length(o.log2_inv_eps, dethost::prime_set_size(bits), logl_H);
      if (kET < 0) kET = INT64_MAX;                 // lemma not applicable: certify only
      for (size_t i = from; i < cra_p.size() && !done; i++) {
        const uint32_t p = cra_p[i];
        const uint64_t km = K.mod_small(p);
        if (km == 0) continue;                       // p | K: skip this prime
        if (crt.count > 0 && crt.M.mod_small(p) == 0) continue;   // (a prime drawn twice)
        const uint64_t kinv = dethost::powmod64(km, p - 2, p);
        crt.add(p, (uint32_t)dethost::mulmod64(cra_r[i], kinv, p));
        if ((double)(crt.M.bit_length() - 1) >= 1.0 + log2_HK + 1.0) done = true;
        else if (!o.certify && crt.same >= kET) {
          done = true;
          rep.early_terminated = 1;
        }
      }
      return kET;
    };
    auto cra_run = [&](double budget_ms) -> det_status {
      const double tb = now_ms();
      restart_crt();
      const double th0 = now_ms();
      int64_t kET = feed(0);
      t_host += now_ms() - th0;
      while (!done && now_ms() - tb < budget_ms) {
        const double log2_HK = std::max(0.0, bd.log2_h - (double)(K.bit_length() - 1));
        const double need = (1.0 + log2_HK + 1.0 - (double)(crt.M.bit_length() - 1)) / log2_l;
        int64_t batch = std::min<int64_t>(std::max<int64_t>((int64_t)ceil(need) + 1, 4), 512);
        if (!o.certify) batch = std::min<int64_t>(batch, std::max<int64_t>(2 * std::min<int64_t>(kET, 64), 8));
        std::vector<uint32_t> ps(batch), rs(batch);
        for (auto& q : ps) q = samp.next();
        const double t0 = now_ms();
        TRY(residues_core(c, c->ws[0], dA, dlda, (int)n, ps.data(), batch, rs.data(), o.path));
        t_lu_ms += now_ms() - t0;
        lu_primes += (double)batch;
        rep.et_rounds++;
        const size_t from = cra_p.size();
        cra_p.insert(cra_p.end(), ps.begin(), ps.end());
        cra_r.insert(cra_r.end(), rs.begin(), rs.end());
        const double th = now_ms();
        kET = feed(from);
        t_host += now_ms() - th;
      }
      return DET_OK;
    };
    auto take_batch1 = [&]() -> det_status {       // the background batch, once
      cra_join.join();
      TRY(cra_st);
      TRY(spin_stream(c, c->own2));
      if (cra_def.count) {
        // a prime whose block-pivot LU met an all-zero block column: again
        // with the full pivot search
        bool any = false;
        for (int64_t i = 0; i < cra_def.count; i++) any |= cra_def.flags[i] != 0;
        if (any) {
          c->block_pivot_retries++;
          TRY(residues_core(c, c->ws[1], dA, dlda, (int)n, ps1.data() + cra_def.s0, cra_def.count,
                            hres1 + cra_def.s0, o.path, true, nullptr, false));
        }
      }
      float ms = 0;
      if (hipEventElapsedTime(&ms, c->ev_t0, c->ev_t1) == hipSuccess && ms > 0) {
        t_lu_ms += ms;
        lu_primes += (double)batch1;
      }
      (void)hipGetLastError();
      cra_p.assign(ps1.begin(), ps1.end());
      cra_r.assign(hres1, hres1 + batch1);
      // the lifting primes' residues from the inverse's LU (free extra CRA
      // residues), when its block pivot search found every pivot
      if (solving && st0 == DET_OK && inv_flag0) {
        TRY(spin_event(c, c->ev_det));
        bool ok = true;
        for (int z = 0; z < np; z++) ok &= inv_flag0[z] == 0;
        if (ok) {
          cra_p.insert(cra_p.begin(), dps0, dps0 + np);
          cra_r.insert(cra_r.begin(), hdet0, hdet0 + np);
        }
      }
      rep.et_rounds = 1;
      return DET_OK;
    };

    // ---------------- LIF: the solvings of Alg. 4.1 (Section 2.2; the
    // extended bonus of Section 3.2 from the second one on)
    for (int pass = 0; pass < 2 && solving; pass++) {
      // one set of primes and inverses for every solving (pass 0 starts with
      // the inverse enqueued above)
      uint32_t dps[detk::LIFT_MAX_PRIMES] = {0, 0, 0, 0};
      det_status st = DET_E_SINGULAR_MOD_P;
      const int32_t* inv_flag = nullptr;
      int tries = 0;
      if (pass == 0) {
        memcpy(dps, dps0, sizeof(dps));
        st = st0;
        inv_flag = inv_flag0;
        tries = 1;
      }
      for (; tries < 2 && st == DET_E_SINGULAR_MOD_P; tries++) {
        draw_dixon(dps);
        st = inverse_mod_primes(c, dA, dlda, (int)n, dps, np, nullptr);
      }
      if (st != DET_OK && st != DET_E_SINGULAR_MOD_P) return st;
      bool redo = false;
      if (st == DET_OK) {                            // else det is probably 0: CRA alone
        // lifting length from the bounds of every combination R_a . x_h:
        // numerators |.| <= sum(R_a) H_col ||b|| / min_j ||a_j|| (Cramer,
        // R entries < 2^16, b entries < beta), denominators <= H; with np
        // primes, k digits of each (prod p_z^k > 2^(Nbits + Dbits + 2))
        const double log2N = log2(65535.0 * (double)n) + bd.log2_hcol +
                             0.5 * log2(std::max(1.0, (double)n * (double)beta * (double)beta)) -
                             bd.log2_min_col + 1e-6;
        const int64_t Nbits = (int64_t)ceil(log2N), Dbits = (int64_t)ceil(bd.log2_h + 1e-6);
        double log2P = 0;
        for (int z = 0; z < np; z++) log2P += log2((double)dps[z]);
        const int64_t k = (int64_t)ceil((double)(Nbits + Dbits + 2) / log2P) + 1;
        const int64_t npad = lift_pad((int)n);
        TRY(ensure(c, c->digits, (size_t)i_max * np * k * n * sizeof(uint32_t)));
        TRY(ensure(c, c->cvec, (size_t)i_max * npad * sizeof(uint32_t)));
        TRY(ensure(c, c->comb, (size_t)i_max * i_max * np * k * sizeof(uint64_t)));
        dethost::PadicCrt crt_p;
        bool crt_ready = false;
        uint32_t* dig = (uint32_t*)c->digits.p;
        std::vector<uint32_t> R((size_t)i_max * npad, 0);
        BigInt K_prev = BigInt::from_i64(1);
        // every launch of the background batch is on own2 before the first
        // lifting waits for it (the cooperative lifting needs its workgroups
        // resident together)
        cra_join.join();
        TRY(cra_st);
        for (int i = 1; i <= i_max; i++) {
          const double ts0 = now_ms();
          std::vector<int64_t> b(n);
          for (int64_t j = 0; j < n; j++) b[j] = (int64_t)(dethost::splitmix64(rng) % (uint64_t)beta);
          // a fresh random i x n matrix R for the i x i combinations R_a . x_h
          for (int a = 0; a < i; a++)
            for (int64_t j = 0; j < n; j++)
              R[(size_t)a * npad + j] = 1 + (uint32_t)(dethost::splitmix64(rng) % 65535u);
          const int* lift_err = nullptr;
          // Before the first lifting is launched (its preparation queued),
          // the background batch is taken: with the adaptive loop, when its
          // residues already end the CRA on det itself (K = 1: early
          // termination, Alg. 2.1, or the bound 2H), no solving is needed
          // and none is launched (Alg. 4.1 stops when the CRA has
          // terminated).  The host has then waited for the batch, so the
          // lifting need not wait for its stream.
          bool cra_done_first = false, inverse_failed = false;
          const PreLaunch pre = [&](bool* skip) -> det_status {
            TRY(take_batch1());
            batch1_taken = true;
            if (o.adaptive && K.cmp(BigInt::from_i64(1)) == 0) {
              restart_crt();
              const double th = now_ms();
              feed(0);
              t_host += now_ms() - th;
              if (done) *skip = cra_done_first = true;
            }
            // the inverse's block pivot flags are back (take_batch1 waited
            // for them): a block column without a non-zero entry means the
            // inverse must be redone with the full search, so this lifting
            // is not launched at all
            if (!*skip && inv_flag && pass == 0) {
              for (int z = 0; z < np; z++) inverse_failed |= inv_flag[z] != 0;
              if (inverse_failed) *skip = true;
            }
            return DET_OK;
          };
          uint32_t* dig_i = dig + (size_t)(i - 1) * np * k * n;
          if (grid3 > 0)
            TRY(lift3_multi(c, grid3, dA, dlda, (int)n, bd.amax, b.data(), 1, dps, np, k, dig_i,
                            false, &lift_err, batch1_taken ? nullptr : &pre));
          else
            TRY(lift(c, dA, dlda, (int)n, bd.amax, b.data(), dps[0], k, dig_i, nullptr, nullptr,
                     false, &lift_err, batch1_taken ? nullptr : &pre));
          if (cra_done_first) {
            HIPCHK(hipStreamSynchronize(c->st));    // (the queued preparation ends)
            break;
          }
          if (inverse_failed) {                     // see pass above
            HIPCHK(hipStreamSynchronize(c->st));
            inv_flag = nullptr;
            c->block_pivot_retries++;
            // before the inverse is redone (with the full search) and a
            // solving run, the CRA on det itself resumes for about that
            // long: a small determinant ends there (Alg. 4.1 stops when the
            // CRA has terminated)
            if (o.adaptive && K.cmp(BigInt::from_i64(1)) == 0) {
              TRY(cra_run(now_ms() - tl0));
              if (done) break;
            }
            redo = true;
            break;
          }
          HIPCHK(hipMemcpyAsync(c->cvec.p, R.data(), (size_t)i * npad * sizeof(uint32_t),
                                hipMemcpyHostToDevice, c->st));
          for (int h = 0; h < i; h++)
            for (int a = 0; a < i; a++)
              for (int z = 0; z < np; z++)
                HIPCHK(detk::launch_comb_digits(
                    dig + ((size_t)h * np + z) * k * n, k, (int)n,
                    (const uint32_t*)c->cvec.p + (size_t)a * npad,
                    (uint64_t*)c->comb.p + (((size_t)h * i + a) * np + z) * k, c->st));
          // (into pinned memory: a copy into pageable memory would hold the
          // host until the lifting has ended)
          const size_t ncomb = (size_t)i * i * np * k;
          TRY(ensure_pin(c, c->hcomb, ncomb * sizeof(uint64_t), c->st));
          uint64_t* comb = (uint64_t*)c->hcomb.p;
          HIPCHK(hipMemcpyAsync(comb, c->comb.p, ncomb * sizeof(uint64_t),
                                hipMemcpyDeviceToHost, c->st));
          if (!crt_ready) {
            // the remaindering constants of the primes, while the device lifts
            const double th = now_ms();
            if (!crt_p.setup(dps, np, k)) return fail(c, DET_E_INVALID, "lifting primes not distinct");
            crt_ready = true;
            t_host += now_ms() - th;
          }
          TRY(spin_stream(c, c->st));
          if (inv_flag) {
            bool bad = false;
            for (int z = 0; z < np; z++) bad |= inv_flag[z] != 0;
            inv_flag = nullptr;
            if (bad) {                               // see pass above
              c->block_pivot_retries++;
              redo = true;
              break;
            }
          }
          if (lift_err && *lift_err)
            return fail(c, DET_E_DEVICE, "lifting: a wait for another workgroup's digits timed out");
          rep.lifting_steps += k;
          const double th0 = now_ms();
          BigInt sv, pi;
          const int64_t failed =
              dethost::extended_bonus_host(comb, i, k, dps, np, Nbits, Dbits, &crt_p, sv, pi);
          K = BigInt::div_exact(K * sv, BigInt::gcd(K, sv));
          K = BigInt::div_exact(K * pi, BigInt::gcd(K, pi));
          if (i >= 2) rep.bonus_factors = failed ? -i : i;
          t_host += now_ms() - th0;
          const double t_solve = now_ms() - ts0;
          rep.solvings = i;
          rep.t_solve_ms = t_solve;
          if (!batch1_taken) {
            TRY(take_batch1());
            batch1_taken = true;
          }
          if (!o.adaptive) continue;                 // exactly i_max solvings, then the CRA
          // resume the CRA on det/K for at most the time of one solving
          TRY(cra_run(t_solve));
          if (done) break;
          if (i >= 2) {
            // Section 5.3: the factor gained by this solving against what
            // the CRA would have gained in its time
            const double gain = (double)(K.bit_length() - K_prev.bit_length());
            const double ratio = lu_primes > 0 ? t_solve / (t_lu_ms / lu_primes) : 0.0;
            if (K.cmp(K_prev) == 0 || gain <= ratio * log2_l) {
              rep.timing_switch = K.cmp(K_prev) == 0 ? 0 : 1;
              break;
            }
          }
          K_prev = K;
        }
      }
      if (!redo) break;
    }
    rep.sn_bits = K.bit_length();
    rep.t_lif_ms = now_ms() - tl0;
    if (!batch1_taken) TRY(take_batch1());
    if (!done) TRY(cra_run(INFINITY));
    rep.primes_used = (int64_t)crt.count;
    rep.t_lu_ms = lu_primes > 0 ? t_lu_ms / lu_primes : 0.0;
    rep.t_cra_ms = now_ms() - tc0;
    const double th1 = now_ms();
    BigInt det = crt.r * K;
    t_host += now_ms() - th1;
    rep.t_host_ms = t_host;
    if (report) *report = rep;
    return emit(det);
  } catch (const std::exception& e) {
    return fail(c, DET_E_NOMEM, e.what());
  } catch (...) {
    return fail(c, DET_E_INVALID, "unexpected error");
  }
}

}  // extern "C"
