// Launchers of the gfx950 kernels (host-callable, all asynchronous on `st`).
// Every launcher returns the HIP error of the launch.  Shapes and pointers
// are checked by the caller (the C-ABI layer) before any launch.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modp.hpp"

namespace detk {

hipError_t launch_residues(const int64_t* A, int64_t lda, int n, int ncols, int32_t* W, int64_t ldw,
                           int64_t slab, const Modulus* mods, int nitems, hipStream_t st);
hipError_t launch_panel(int32_t* W, int64_t ldw, int64_t slab, int n, int j0, int pb, int pbw,
                        const Modulus* mods, int32_t* piv, int64_t piv_stride, int32_t* flags,
                        int32_t* Linv, int32_t* Uinv, int kc, int nitems, int ncols_sw,
                        hipStream_t st);
// One LU step's update of the trailing block in one launch (U12 from L11^{-1}
// A12 per column tile, stored by the last reader when cnt != null; A22 -=
// L21 U12); the panel's swaps already applied (launch_panel with ncols_sw).
// Uinv != null: the panel factored only its diagonal block, and L21 is formed
// as A21 U11^{-1} inside the update (U11^{-1} from the panel, ldt x ldt).
// next_pb > 0 (needs Uinv != null, ldt == 32): the launch also factors the
// next diagonal block, at (j0 + pb, j0 + pb) with width next_pb, as
// launch_diag_block would, into next_Linv / next_Uinv (other buffers than
// Linv / Uinv), piv and flags.
hipError_t launch_lu_update(int32_t* W, int64_t slab, int64_t ldw, int j0, int pb, int M, int N,
                            const int32_t* Linv, int ldt, const int32_t* Uinv,
                            const Modulus* mods, int kc4, unsigned* cnt, int cnt_stride,
                            int nitems, hipStream_t st, int next_pb = 0,
                            int32_t* next_Linv = nullptr, int32_t* next_Uinv = nullptr,
                            int32_t* piv = nullptr, int64_t piv_stride = 0,
                            int32_t* flags = nullptr);
int panel_width_for(int m);
// The pb x pb diagonal block at (j0, j0) of every item (pb <= 32) factored
// without pivot search below it: U11 into W, L11^{-1} and U11^{-1} dense
// 32 x 32 (Linv, Uinv + z * 1024), piv = identity on the block, flags[z] = 1
// when a pivot is 0 mod p.
hipError_t launch_diag_block(int32_t* W, int64_t ldw, int64_t slab, int j0, int pb,
                             const Modulus* mods, int32_t* piv, int64_t piv_stride, int32_t* flags,
                             int32_t* Linv, int32_t* Uinv, int nitems, hipStream_t st);
hipError_t launch_swaps(int32_t* W, int64_t ldw, int64_t slab, int j0, int pb, const int32_t* piv,
                        int64_t piv_stride, int c0a, int c1a, int c0b, int c1b, int nitems,
                        hipStream_t st);
hipError_t launch_tri_inv(const int32_t* W, int64_t ldw, int64_t slab, int k0, int kb,
                          const Modulus* mods, int32_t* Tinv, int ldt, int nitems, hipStream_t st);
hipError_t launch_trsm_apply(int32_t* W, int64_t slab, int64_t ldw, int r0, int kb, int c0, int N,
                             const int32_t* Tinv, int ldt, const Modulus* mods, int kc4,
                             const int32_t* piv, int64_t piv_stride, int sw_j0, int sw_pb,
                             int nitems, hipStream_t st);
hipError_t launch_gemm_f64(int32_t* W, int64_t slab, int64_t offC, int64_t offA, int64_t offB,
                           int64_t ldw, int M, int N, int K, const Modulus* mods, int kc4,
                           int nitems, hipStream_t st);
// Limb planes (3 x Rp x Kp int8 per item, zero-padded) of an M x K block or
// of a K x N block transposed; p < 2^23.
hipError_t launch_split(const int32_t* W, int64_t slab, int64_t off, int64_t ldw, int rows, int K,
                        int Kp, int64_t Rp, int transpose, int8_t* P, int64_t pslab, int nitems,
                        hipStream_t st);
// C -= A B mod p from limb planes (K padded to Kp <= 43690).
hipError_t launch_gemm_i8(int32_t* W, int64_t slab, int64_t offC, int64_t ldw, int M, int N,
                          const int8_t* PA, const int8_t* PB, int64_t pslabA, int64_t pslabB,
                          int64_t MpA, int64_t NpB, int Kp, const Modulus* mods, int nitems,
                          hipStream_t st);
hipError_t launch_det_finalize(const int32_t* W, int64_t ldw, int64_t slab, int n,
                               const int32_t* piv, int64_t piv_stride, const int32_t* flags,
                               const Modulus* mods, uint32_t* out, int nitems, hipStream_t st);
// Cu[z] (n x n, canonical) = the n x n block at column col0 of item z, for
// the nitems items at W + z * slab.
hipError_t launch_extract_inverse(const int32_t* W, int64_t slab, int64_t ldw, int64_t col0, int n,
                                  const Modulus* mods, uint32_t* Cu, int nitems, hipStream_t st);
// C <op> A B (mod p) on int32 centred residues within one slab per item
// (op 0: C -= AB, 1: C += AB, 2: C = AB, 3: C = -AB); upper_a: A is upper
// triangular (a row tile starts K at its row).  Items: nitems x nouter, item
// (zo, zi) at W + zo * slab_outer + zi * slab, with modulus mods[zo] when
// mod_by_outer, else mods[zo * nitems + zi].
hipError_t launch_gemm_mod(int32_t* W, int64_t slab, int64_t offC, int64_t offA, int64_t offB,
                           int64_t ldw, int M, int N, int K, const Modulus* mods, int kc4, int op,
                           bool upper_a, int nitems, hipStream_t st, int nouter = 1,
                           int64_t slab_outer = 0, bool mod_by_outer = false);
// The 32 x 32 diagonal-block inverses (panel-major: panel q of item z at
// (q * nitems + z) * 1024) onto the diagonal of the n x n region at offV of
// each item.
hipError_t launch_place_diag(int32_t* W, int64_t slab, int64_t ldw, int64_t offV, int n,
                             const int32_t* uinv, int nitems, hipStream_t st);

// Dixon lifting (dixon_kernels.hip).
hipError_t launch_lift_x(const uint32_t* Cu, const uint32_t* rp, int n, uint32_t p,
                         uint32_t* xout, hipStream_t st);
hipError_t launch_lift_r(const int32_t* Ai, const uint32_t* x, int64_t* r, uint32_t* rp, int n,
                         uint32_t p, uint64_t pinv64, const uint32_t* cvec, uint64_t* comb,
                         hipStream_t st);

// Cooperative form: all k steps in one launch (grid from lift_persistent_grid,
// 0 when the device cannot run it).  bar and err must be zero at launch.
int lift_persistent_grid(int device, int n);
hipError_t launch_lift_persistent(int grid, const uint32_t* Cu, const int32_t* Ai, int64_t* r,
                                  uint32_t* rp, uint32_t* xbuf, int n, uint32_t p, uint64_t pinv64,
                                  int64_t k, uint32_t* digits, const uint32_t* cvec,
                                  uint64_t* comb, unsigned* bar, int* err, hipStream_t st);

// Lifting modulo p^2 (two base-p digits per step, n <= 1024): the Hensel
// step C1 = digit plane of A^{-1} mod p^2 (E: n x n scratch), then all steps.
hipError_t launch_hensel(const int32_t* Ai, const uint32_t* Cu, uint32_t* E, uint32_t* C1, int n,
                         uint32_t p, hipStream_t st);
// Lifting modulo p^3 in FP64 (p < 2^25, n ||A|| p < 2^53, n <= 2048): Hensel planes
// C1, C2 of A^{-1} mod p^3 from C0 = A^{-1} mod p (E: n x n FP64 scratch),
// then all steps in one cooperative launch, three digits per step.
int lift3_grid(int device, int n);    // 0: the three-plane form does not apply
// liftings of order n that one launch can run side by side (1 .. LIFT_MAX_PRIMES;
// 0 when the three-plane form does not apply)
int lift3_max_primes(int device, int n);
// comb[i] = cvec . digits[i] for k digit vectors of length n (after a lifting)
hipError_t launch_comb_digits(const uint32_t* digits, int64_t k, int n, const uint32_t* cvec,
                              uint64_t* comb, hipStream_t st);
// Words of the vectors that the three-plane lifting passes between its
// workgroups: a 25-bit digit field (two's complement for the balanced digits
// of r) under a 7-bit tag, the step number mod 127; tag 127 (an all-ones
// word) marks a word not yet written.  r of step 0 goes in with tag 0.
constexpr uint32_t LIFT3_DIGIT_MASK = 0x1FFFFFFu;
// Largest magnitude that three signed int8 limbs hold on both sides
// (limb_word): the int8 paths need every operand value within it.
constexpr int32_t LIMB3_MAX = 0x7F7F7F;

// Several liftings side by side, one per prime (Section 6: p-adic liftings
// in parallel, each with fewer steps): the primes of one launch, with their
// reciprocals.
constexpr int LIFT_MAX_PRIMES = 4;
struct PrimeSet {
  uint32_t p[LIFT_MAX_PRIMES];
  double pinv[LIFT_MAX_PRIMES];
};
// The Hensel planes for np primes at once: C0, E, C1, C2 hold np n x n
// matrices each (prime z at offset z n^2); Ai is shared.
hipError_t launch_hensel_f64(const int32_t* Ai, const uint32_t* C0, double* E, uint32_t* C1,
                             uint32_t* C2, int n, const uint32_t* primes, int np, hipStream_t st);
// The same planes from int8 MFMA on three limbs of every operand: needs
// |a_ij| <= 0x7F7F7F and every p <= 2 * 0x7F7F7F + 1; `planes` is device
// scratch of hensel_i8_scratch(n, np) bytes.
size_t hensel_i8_scratch(int n, int np);
hipError_t launch_hensel_i8(const int32_t* Ai, const uint32_t* C0, double* E, uint32_t* C1,
                            uint32_t* C2, int n, const uint32_t* primes, int np, int8_t* planes,
                            hipStream_t st);
// rv, xv: n x nrhs x 4 words, the digit vectors passed between workgroups (r
// of step 0 in rv under tag 0, xv filled with all-ones words before the
// launch); r: n x nrhs (row-major); digits of right-hand side h at
// digits + h * dig_rhs_stride (kd x n).  nrhs <= LIFT3_MAX_RHS right-hand
// sides share one launch.  With np > 1 primes, np liftings run side by side,
// `grid` workgroups each: prime z has its planes at C* + z n^2, its r at
// r + z n nrhs, its vectors at rv, xv + 4 z n nrhs and its digits at digits +
// z * dig_prime_stride; Ai and err are shared.
constexpr int LIFT3_MAX_RHS = 2;
int lift3_max_rhs(int n);             // right-hand sides one launch takes at order n
hipError_t launch_lift_resident3(int grid, const uint32_t* C0, const uint32_t* C1,
                                 const uint32_t* C2, const int32_t* Ai, int64_t* r, uint32_t* rv,
                                 uint32_t* xv, int n, int nrhs, const uint32_t* primes, int np,
                                 int64_t kd, uint32_t* digits, int64_t dig_rhs_stride,
                                 int64_t dig_prime_stride, int* err, hipStream_t st);
hipError_t launch_lift_resident2(int grid, const uint32_t* C0, const uint32_t* C1,
                                 const int32_t* Ai, int64_t* r, uint32_t* rp0, uint32_t* rp1,
                                 uint32_t* xb0, uint32_t* xb1, int n, uint32_t p, uint64_t pinv64,
                                 int64_t kd, uint32_t* digits, const uint32_t* cvec,
                                 uint64_t* comb, unsigned* bar, int* err, hipStream_t st);

// Persistent LU over a work queue (batch_kernels.hip).  One item is one
// (matrix, prime) pair: A device row-major int64 with leading dimension lda,
// order n <= lu_queue_max_n(variant), odd prime p < 2^26; the result
// det(A) mod p goes to out[out_index].
struct LuItem {
  const int64_t* A;
  int64_t lda;
  int32_t n;
  uint32_t p;
  int32_t out_index;
  int32_t pad;
};
// Kernel variants, all for orders up to 512: panel width 32 (one workgroup
// per CU), panel width 16 (one per CU), panel width 16 compiled for two
// workgroups per CU (registers capped at 256 a lane).
enum { LU_QUEUE_PB32 = 1, LU_QUEUE_PB16 = 2, LU_QUEUE_PB16X2 = 3 };
int lu_queue_max_n(int variant);
int lu_queue_blocks_per_cu(int variant);          // resident workgroups per CU at most
int64_t lu_queue_aux_stride();                    // int32 per workgroup in `aux`
// Slab stride (int32) per workgroup for orders up to nmax.
inline int64_t lu_queue_ws_stride(int nmax) {
  return ((int64_t)(nmax + 63) / 64 * 64 + 4) * nmax;
}
// next[0 .. count) = 0 (a kernel, so that it can be captured in a graph).
hipError_t launch_queue_reset(unsigned* next, int count, hipStream_t st);
// `grid` workgroups take items[next[0]++] until the queue is empty; ws: grid
// slabs of ws_stride int32; aux: grid x lu_queue_aux_stride() int32.
hipError_t launch_lu_queue(int variant, int grid, const LuItem* items, int nitems, unsigned* next,
                           int32_t* ws, int64_t ws_stride, int32_t* aux, uint32_t* out,
                           hipStream_t st);

hipError_t launch_pack_i32(const int64_t* A, int64_t lda, int n, int32_t* Ai, hipStream_t st);
hipError_t launch_norms(const int64_t* A, int64_t lda, int n, double* out2n, double* amax,
                        hipStream_t st);
// The same over a grid of 64 x 64 blocks (one launch for the partial sums,
// one to add them); part: norms_scratch(n) doubles of device scratch.
size_t norms_scratch(int n);
hipError_t launch_norms_wide(const int64_t* A, int64_t lda, int n, double* out2n, double* amax,
                             double* part, hipStream_t st);

// Configure dynamic-LDS limits once per device.
hipError_t configure_kernels();

}  // namespace detk
