// C-ABI of the library (include/det.h): contexts, the blocked LU driver,
// det_mod_primes, dixon_lift and det_introspective.  Every device step runs
// in the HIP kernels of lu_kernels.hip and dixon_kernels.hip; the host keeps
// prime sampling, Chinese remaindering with early termination, the p-adic to
// integer conversion, rational reconstruction and the final product.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <exception>
#include <string>
#include <vector>

#include "../../include/det.h"
#include "../../include/det_host.h"
#include "bigint.hpp"
#include "host_numerics.hpp"
#include "kernels.hpp"

using dethost::BigInt;
using detk::Modulus;

namespace {

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

constexpr int NB_OUTER = 128;      // outer block (trailing-update depth K)
constexpr int TINV_LD = 128;       // leading dimension of the outer triangular inverses
constexpr int MAX_N = 4096;

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct det_ctx {
  int device = 0;
  size_t budget = 0;
  size_t held = 0;
  hipStream_t own = nullptr;
  hipStream_t st = nullptr;
  std::string err;
  DevBuf W, piv, flags, mods, linv, tinv, limbA, limbB, res, Adev, norms, amax;
  DevBuf Cu, Ai, r, rp, x, digits, comb, cvec;
  // kernel timing (det_profile_select / det_profile_read)
  int prof_kind = 0;
  int64_t prof_launches = 0;
  double prof_bytes = 0, prof_ops = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending;
  std::vector<hipEvent_t> ev_pool;
};

namespace {

det_status fail(det_ctx* c, det_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(c, DET_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Grow-only device buffer; the previous contents are not kept.
det_status ensure(det_ctx* c, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (b.cap >= bytes) return DET_OK;
  if (c->budget && c->held - b.cap + bytes > c->budget)
    return fail(c, DET_E_NOMEM, "device workspace would exceed the context's HBM budget");
  HIPCHK(hipStreamSynchronize(c->st));
  if (b.p) {
    HIPCHK(hipFree(b.p));
    c->held -= b.cap;
    b.p = nullptr;
    b.cap = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return fail(c, DET_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  b.cap = bytes;
  c->held += bytes;
  return DET_OK;
}

#define TRY(expr)                     \
  do {                                \
    det_status s_ = (expr);           \
    if (s_ != DET_OK) return s_;      \
  } while (0)

// Brackets one launch with HIP events when its kernel class is the selected
// one; the counts are the launcher's algorithmic bytes and operations.
struct ProfScope {
  det_ctx* c;
  hipEvent_t e1 = nullptr;
  ProfScope(det_ctx* ctx, int kind, double bytes, double ops) : c(ctx) {
    if (c->prof_kind != kind) return;
    hipEvent_t e0 = take(), e = take();
    if (!e0 || !e) return;
    if (hipEventRecord(e0, c->st) != hipSuccess) return;
    e1 = e;
    c->prof_pending.push_back({e0, e1});
    c->prof_launches++;
    c->prof_bytes += bytes;
    c->prof_ops += ops;
  }
  ~ProfScope() {
    if (e1) (void)hipEventRecord(e1, c->st);
  }
  hipEvent_t take() {
    if (!c->ev_pool.empty()) {
      hipEvent_t e = c->ev_pool.back();
      c->ev_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice;
}

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

// ------------------------------------------------------------------ LU driver
struct LuJob {
  int n = 0;          // rows (and columns of A)
  int ncols = 0;      // n, or 2n for [A | I]
  int nitems = 0;     // batch items (one prime each)
  int64_t ldw = 0, slab = 0;
  bool int8 = false;
  uint32_t pmax = 0;
};

int panel_width(int n) { return n <= 2048 ? 32 : 16; }

// Blocked right-looking LU of every item (see lu_kernels.hip for the data
// layout).  W, piv, flags, mods must already hold the residues and moduli.
det_status lu_factor(det_ctx* c, const LuJob& J) {
  const int n = J.n, ncols = J.ncols, nit = J.nitems;
  const int64_t ldw = J.ldw, slab = J.slab;
  const int PB = panel_width(n);
  const int kc = exact_chunk(J.pmax);
  const int kc4 = std::max(1, kc / 4);
  int32_t* W = (int32_t*)c->W.p;
  int32_t* piv = (int32_t*)c->piv.p;
  int32_t* flags = (int32_t*)c->flags.p;
  const Modulus* mods = (const Modulus*)c->mods.p;
  TRY(ensure(c, c->linv, (size_t)nit * PB * PB * sizeof(int32_t)));
  TRY(ensure(c, c->tinv, (size_t)nit * TINV_LD * TINV_LD * sizeof(int32_t)));
  int32_t* linv = (int32_t*)c->linv.p;
  int32_t* tinv = (int32_t*)c->tinv.p;
  int Kp = 0;
  int64_t pslabA = 0, pslabB = 0;
  if (J.int8) {
    Kp = NB_OUTER;                                  // multiple of 64
    pslabA = 3LL * n * Kp;
    pslabB = 3LL * ncols * Kp;
    TRY(ensure(c, c->limbA, (size_t)nit * pslabA));
    TRY(ensure(c, c->limbB, (size_t)nit * pslabB));
  }
  hipStream_t st = c->st;
  for (int k0 = 0; k0 < n; k0 += NB_OUTER) {
    const int kb = std::min(NB_OUTER, n - k0);
    for (int j0 = k0; j0 < k0 + kb; j0 += PB) {
      const int pb = std::min(PB, k0 + kb - j0);
      {
        const double m = n - j0;
        ProfScope ps(c, DET_KERNEL_PANEL, 8.0 * m * pb * nit, m * pb * pb * (double)nit);
        HIPCHK(detk::launch_panel(W, ldw, slab, n, j0, pb, PB, mods, piv, n, flags, linv, nit, st));
      }
      HIPCHK(detk::launch_swaps(W, ldw, slab, j0, pb, piv, n, k0, j0, j0 + pb, ncols, nit, st));
      const int rest = k0 + kb - (j0 + pb);
      if (rest > 0) {
        {
          ProfScope ps(c, DET_KERNEL_TRSM, (8.0 * pb * rest + 4.0 * pb * pb) * nit,
                       2.0 * pb * pb * rest * nit);
          HIPCHK(detk::launch_trsm_apply(W, slab, ldw, j0, pb, j0 + pb, rest, linv, PB, mods, kc4,
                                         nit, st));
        }
        {
          const double M = n - (j0 + pb);
          ProfScope ps(c, DET_KERNEL_GEMM_F64, 4.0 * (M * pb + pb * rest + 2.0 * M * rest) * nit,
                       2.0 * M * rest * pb * nit);
          HIPCHK(detk::launch_gemm_f64(W, slab, (int64_t)(j0 + pb) * ldw + j0 + pb,
                                       (int64_t)(j0 + pb) * ldw + j0, (int64_t)j0 * ldw + j0 + pb,
                                       ldw, n - (j0 + pb), rest, pb, mods, kc4, nit, st));
        }
      }
    }
    const int right = ncols - (k0 + kb);
    if (right <= 0) continue;
    {
      ProfScope ps(c, DET_KERNEL_TRI_INV, 8.0 * kb * kb * nit, (double)kb * kb * kb / 3.0 * nit);
      HIPCHK(detk::launch_tri_inv(W, ldw, slab, k0, kb, 0, mods, tinv, TINV_LD, kc, nit, st));
    }
    {
      ProfScope ps(c, DET_KERNEL_TRSM, (8.0 * kb * right + 4.0 * kb * kb) * nit,
                   2.0 * kb * kb * right * nit);
      HIPCHK(detk::launch_trsm_apply(W, slab, ldw, k0, kb, k0 + kb, right, tinv, TINV_LD, mods,
                                     kc4, nit, st));
    }
    const int M = n - (k0 + kb);
    if (M <= 0) continue;
    const int64_t offC = (int64_t)(k0 + kb) * ldw + k0 + kb;
    const int64_t offA = (int64_t)(k0 + kb) * ldw + k0;
    const int64_t offB = (int64_t)k0 * ldw + k0 + kb;
    if (J.int8) {
      HIPCHK(detk::launch_split(W, slab, offA, ldw, M, kb, Kp, 0, (int8_t*)c->limbA.p, pslabA, nit,
                                st));
      HIPCHK(detk::launch_split(W, slab, offB, ldw, right, kb, Kp, 1, (int8_t*)c->limbB.p, pslabB,
                                nit, st));
      ProfScope ps(c, DET_KERNEL_GEMM_I8,
                   (3.0 * Kp * (M + right) + 8.0 * M * right) * nit,
                   18.0 * M * right * kb * nit);
      HIPCHK(detk::launch_gemm_i8(W, slab, offC, ldw, M, right, (const int8_t*)c->limbA.p,
                                  (const int8_t*)c->limbB.p, pslabA, pslabB, Kp, mods, nit, st));
    } else {
      ProfScope ps(c, DET_KERNEL_GEMM_F64, 4.0 * ((double)M * kb + (double)kb * right + 2.0 * M * right) * nit,
                   2.0 * M * right * kb * nit);
      HIPCHK(detk::launch_gemm_f64(W, slab, offC, offA, offB, ldw, M, right, kb, mods, kc4, nit,
                                   st));
    }
  }
  return DET_OK;
}

// Back substitution U X = Y on [U | Y] (one item): X = U^{-1} Y = A^{-1} mod p.
det_status back_substitute(det_ctx* c, const LuJob& J) {
  const int n = J.n;
  const int kc = exact_chunk(J.pmax);
  const int kc4 = std::max(1, kc / 4);
  int32_t* W = (int32_t*)c->W.p;
  const Modulus* mods = (const Modulus*)c->mods.p;
  int32_t* tinv = (int32_t*)c->tinv.p;
  const int nblk = (n + NB_OUTER - 1) / NB_OUTER;
  for (int bi = nblk - 1; bi >= 0; bi--) {
    const int k0 = bi * NB_OUTER, kb = std::min(NB_OUTER, n - k0);
    HIPCHK(detk::launch_tri_inv(W, J.ldw, J.slab, k0, kb, 1, mods, tinv, TINV_LD, kc, 1, c->st));
    HIPCHK(detk::launch_trsm_apply(W, J.slab, J.ldw, k0, kb, n, n, tinv, TINV_LD, mods, kc4, 1,
                                   c->st));
    if (k0 > 0)
      HIPCHK(detk::launch_gemm_f64(W, J.slab, n, k0, (int64_t)k0 * J.ldw + n, J.ldw, k0, n, kb,
                                   mods, kc4, 1, c->st));
  }
  return DET_OK;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

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
  TRY(ensure(c, c->norms, (size_t)2 * n * sizeof(double)));
  TRY(ensure(c, c->amax, (size_t)n * sizeof(double)));
  HIPCHK(detk::launch_norms(dA, dlda, (int)n, (double*)c->norms.p, (double*)c->amax.p, c->st));
  std::vector<double> h(2 * n), am(n);
  HIPCHK(hipMemcpyAsync(h.data(), c->norms.p, 2 * n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(am.data(), c->amax.p, n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  double amax = 0;
  for (double v : am) amax = std::max(amax, v);
  if (amax >= 2147483648.0) return fail(c, DET_E_OVERFLOW, "matrix entry with |a_ij| >= 2^31");
  std::vector<double> cols(h.begin(), h.begin() + n), rows(h.begin() + n, h.end());
  *b = dethost::bounds_from_sums(cols, rows, amax);
  return DET_OK;
}

// Modular determinants of a staged device matrix for a list of primes, in
// batches bounded by the workspace.  Path already validated.
det_status residues_core(det_ctx* c, const int64_t* dA, int64_t dlda, int n,
                         const uint32_t* primes, int64_t np, uint32_t* out, bool int8) {
  if (np == 0) return DET_OK;
  if (n == 0) {
    for (int64_t i = 0; i < np; i++) out[i] = 1 % primes[i];
    return DET_OK;
  }
  LuJob J;
  J.n = n;
  J.ncols = n;
  J.ldw = round_up(n, 32);
  J.slab = J.ldw * n;
  J.int8 = int8;
  const size_t per_item = (size_t)J.slab * 4 + 3 * (size_t)(2 * n) * NB_OUTER + TINV_LD * TINV_LD * 4;
  size_t cap_bytes = (size_t)8 << 30;                  // at most 8 GiB of slabs per batch
  if (c->budget) cap_bytes = std::min(cap_bytes, c->budget / 2);
  int64_t bmax = std::max<int64_t>(1, std::min<int64_t>(1024, (int64_t)(cap_bytes / per_item)));
  for (int64_t s0 = 0; s0 < np; s0 += bmax) {
    const int nit = (int)std::min<int64_t>(bmax, np - s0);
    J.nitems = nit;
    J.pmax = 0;
    std::vector<Modulus> hm(nit);
    for (int i = 0; i < nit; i++) {
      hm[i] = modulus_of(primes[s0 + i]);
      J.pmax = std::max(J.pmax, primes[s0 + i]);
    }
    TRY(ensure(c, c->W, (size_t)nit * J.slab * sizeof(int32_t)));
    TRY(ensure(c, c->piv, (size_t)nit * n * sizeof(int32_t)));
    TRY(ensure(c, c->flags, (size_t)nit * sizeof(int32_t)));
    TRY(ensure(c, c->mods, (size_t)nit * sizeof(Modulus)));
    TRY(ensure(c, c->res, (size_t)nit * sizeof(uint32_t)));
    HIPCHK(hipMemcpyAsync(c->mods.p, hm.data(), nit * sizeof(Modulus), hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemsetAsync(c->flags.p, 0, nit * sizeof(int32_t), c->st));
    {
      ProfScope ps(c, DET_KERNEL_RESIDUES, (double)n * n * (8.0 + 4.0 * nit), 0.0);
      HIPCHK(detk::launch_residues(dA, dlda, n, n, (int32_t*)c->W.p, J.ldw, J.slab,
                                   (const Modulus*)c->mods.p, nit, c->st));
    }
    TRY(lu_factor(c, J));
    HIPCHK(detk::launch_det_finalize((const int32_t*)c->W.p, J.ldw, J.slab, n,
                                     (const int32_t*)c->piv.p, n, (const int32_t*)c->flags.p,
                                     (const Modulus*)c->mods.p, (uint32_t*)c->res.p, nit, c->st));
    HIPCHK(hipMemcpyAsync(out + s0, c->res.p, nit * sizeof(uint32_t), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
  }
  return DET_OK;
}

uint64_t inv_mod_2_64(uint64_t p) {
  uint64_t x = p;                         // correct to 3 bits for odd p
  for (int i = 0; i < 5; i++) x *= 2 - p * x;
  return x;
}

// A^{-1} mod p into c->Cu (canonical, n x n), from a staged device matrix.
// Returns DET_E_SINGULAR_MOD_P if p | det(A).
det_status inverse_mod_p(det_ctx* c, const int64_t* dA, int64_t dlda, int n, uint32_t p) {
  LuJob J;
  J.n = n;
  J.ncols = 2 * n;
  J.ldw = round_up(2 * n, 32);
  J.slab = J.ldw * n;
  J.nitems = 1;
  J.pmax = p;
  J.int8 = false;
  Modulus hm = modulus_of(p);
  TRY(ensure(c, c->W, (size_t)J.slab * sizeof(int32_t)));
  TRY(ensure(c, c->piv, (size_t)n * sizeof(int32_t)));
  TRY(ensure(c, c->flags, sizeof(int32_t)));
  TRY(ensure(c, c->mods, sizeof(Modulus)));
  TRY(ensure(c, c->Cu, (size_t)n * n * sizeof(uint32_t)));
  HIPCHK(hipMemcpyAsync(c->mods.p, &hm, sizeof(Modulus), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemsetAsync(c->flags.p, 0, sizeof(int32_t), c->st));
  HIPCHK(detk::launch_residues(dA, dlda, n, 2 * n, (int32_t*)c->W.p, J.ldw, J.slab,
                               (const Modulus*)c->mods.p, 1, c->st));
  TRY(lu_factor(c, J));
  int32_t flag = 0;
  HIPCHK(hipMemcpyAsync(&flag, c->flags.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (flag) return fail(c, DET_E_SINGULAR_MOD_P, "p divides det(A)");
  TRY(back_substitute(c, J));
  HIPCHK(detk::launch_extract_inverse((const int32_t*)c->W.p, J.ldw, n, (const Modulus*)c->mods.p,
                                      (uint32_t*)c->Cu.p, c->st));
  return DET_OK;
}

// k Dixon steps from r_0 = b.  digits_dev: k x n output (may be null when only
// the combinations are wanted); comb_dev: k sums of cvec . x_i (may be null).
det_status lift(det_ctx* c, const int64_t* dA, int64_t dlda, int n, const int64_t* b, uint32_t p,
                int64_t k, uint32_t* digits_dev, const uint32_t* cvec_dev, uint64_t* comb_dev) {
  TRY(ensure(c, c->Ai, (size_t)n * n * sizeof(int32_t)));
  TRY(ensure(c, c->r, (size_t)n * sizeof(int64_t)));
  TRY(ensure(c, c->rp, (size_t)n * sizeof(uint32_t)));
  TRY(ensure(c, c->x, (size_t)n * sizeof(uint32_t)));
  HIPCHK(detk::launch_pack_i32(dA, dlda, n, (int32_t*)c->Ai.p, c->st));
  std::vector<uint32_t> rp0(n);
  for (int j = 0; j < n; j++) {
    int64_t m = b[j] % (int64_t)p;
    rp0[j] = (uint32_t)(m < 0 ? m + p : m);
  }
  HIPCHK(hipMemcpyAsync(c->r.p, b, n * sizeof(int64_t), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(c->rp.p, rp0.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, c->st));
  const uint64_t pinv64 = inv_mod_2_64(p);
  for (int64_t i = 0; i < k; i++) {
    uint32_t* xi = digits_dev ? digits_dev + i * n : (uint32_t*)c->x.p;
    const double nn = (double)n * n;
    {
      ProfScope ps(c, DET_KERNEL_LIFT_X, 4.0 * nn + 8.0 * n, 2.0 * nn);
      HIPCHK(detk::launch_lift_x((const uint32_t*)c->Cu.p, (const uint32_t*)c->rp.p, n, p, xi,
                                 c->st));
    }
    {
      ProfScope ps(c, DET_KERNEL_LIFT_R, 4.0 * nn + 24.0 * n, 2.0 * nn);
      HIPCHK(detk::launch_lift_r((const int32_t*)c->Ai.p, xi, (int64_t*)c->r.p,
                                 (uint32_t*)c->rp.p, n, p, pinv64, cvec_dev,
                                 comb_dev ? comb_dev + i : nullptr, c->st));
    }
  }
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

}  // namespace

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
      hipSetDevice(device) != hipSuccess || hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess ||
      detk::configure_kernels() != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return DET_E_DEVICE;
  }
  c->st = c->own;
  *out = c;
  return DET_OK;
}

void det_ctx_destroy(det_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->st) (void)hipStreamSynchronize(c->st);
  DevBuf* all[] = {&c->W, &c->piv, &c->flags, &c->mods, &c->linv, &c->tinv, &c->limbA, &c->limbB,
                   &c->res, &c->Adev, &c->norms, &c->amax, &c->Cu, &c->Ai, &c->r, &c->rp,
                   &c->x, &c->digits, &c->comb, &c->cvec};
  for (DevBuf* b : all)
    if (b->p) (void)hipFree(b->p);
  for (auto& pr : c->prof_pending) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->own) (void)hipStreamDestroy(c->own);
  delete c;
}

det_status det_ctx_set_stream(det_ctx* c, void* hip_stream) {
  if (!c) return DET_E_INVALID;
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, DET_E_DEVICE, "hipSetDevice failed");
  HIPCHK(hipStreamSynchronize(c->st));
  c->st = hip_stream ? (hipStream_t)hip_stream : c->own;
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
}

det_status det_profile_select(det_ctx* c, det_kernel kind) {
  if (!c || (int)kind < 0 || (int)kind > DET_KERNEL_RESIDUES) return DET_E_INVALID;
  c->prof_kind = (int)kind;
  return DET_OK;
}

det_status det_profile_read(det_ctx* c, int64_t* launches, double* total_ms, double* bytes,
                            double* ops) {
  if (!c) return DET_E_INVALID;
  HIPCHK(hipStreamSynchronize(c->st));
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
    const bool int8 = path == DET_PATH_INT8 || (path == DET_PATH_AUTO && pmax < (1u << 23));
    TRY(check_prime_list(c, primes, nprimes, int8 ? (1u << 23) : (1u << 26)));
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
    return residues_core(c, dA, dlda, (int)n, primes, nprimes, residues, int8);
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
    TRY(lift(c, dA, dlda, (int)n, b, p, k, (uint32_t*)c->digits.p, nullptr, nullptr));
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
    const bool int8 = o.path != DET_PATH_FP64 && o.prime_bits <= 23;
    if (o.prime_bits < 12 || o.prime_bits > (o.path == DET_PATH_INT8 ? 23 : 26))
      return fail(c, DET_E_PRIME_RANGE, "prime_bits out of range");
    det_report rep;
    memset(&rep, 0, sizeof(rep));
    const double t0 = now_ms();
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

    // ---------------- LIF: s~_n from Dixon solvings (Section 2.2)
    BigInt K = BigInt::from_i64(1);
    const double tl0 = now_ms();
    int dixon_bits = 26;
    while (dixon_bits > 12 && (double)n * bd.amax * ldexp(1.0, dixon_bits) >= ldexp(1.0, 62))
      dixon_bits--;
    const int64_t beta = std::max<int64_t>(2, (int64_t)ceil(bd.log2_h));
    if (bd.log2_h > 0 && dixon_bits > 12) {
      dethost::PrimeSampler dsamp(dethost::splitmix64(rng), dixon_bits);
      for (int solve = 0; solve < o.n_rhs; solve++) {
        uint32_t p = 0;
        det_status st = DET_E_SINGULAR_MOD_P;
        for (int tries = 0; tries < 2 && st == DET_E_SINGULAR_MOD_P; tries++) {
          p = dsamp.next();
          st = inverse_mod_p(c, dA, dlda, (int)n, p);
        }
        if (st == DET_E_SINGULAR_MOD_P) break;     // det is probably 0: CRA alone
        if (st != DET_OK) return st;
        // right-hand side b in [0, beta) and the combination vector in [1, 2^16)
        std::vector<int64_t> b(n);
        std::vector<uint32_t> cv(n);
        double csum = 0, b2 = 0;
        for (int64_t j = 0; j < n; j++) {
          b[j] = (int64_t)(dethost::splitmix64(rng) % (uint64_t)beta);
          cv[j] = 1 + (uint32_t)(dethost::splitmix64(rng) % 65535u);
          csum += cv[j];
          b2 += (double)b[j] * (double)b[j];
        }
        // y = c.x = (c.num)/d(x): |c.num| <= sum(c) H_col ||b|| / min_j ||a_j||, d <= H.
        const double log2N = log2(csum) + bd.log2_hcol + 0.5 * log2(std::max(b2, 1.0)) -
                             bd.log2_min_col + 1e-6;
        const double log2D = bd.log2_h + 1e-6;
        const int64_t Nbits = (int64_t)ceil(log2N), Dbits = (int64_t)ceil(log2D);
        const int64_t k = (int64_t)ceil((double)(Nbits + Dbits + 2) / log2((double)p)) + 1;
        TRY(ensure(c, c->cvec, (size_t)n * sizeof(uint32_t)));
        TRY(ensure(c, c->comb, (size_t)k * sizeof(uint64_t)));
        HIPCHK(hipMemcpyAsync(c->cvec.p, cv.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, c->st));
        TRY(lift(c, dA, dlda, (int)n, b.data(), p, k, nullptr, (const uint32_t*)c->cvec.p,
                 (uint64_t*)c->comb.p));
        std::vector<uint64_t> comb(k);
        HIPCHK(hipMemcpyAsync(comb.data(), c->comb.p, k * sizeof(uint64_t), hipMemcpyDeviceToHost, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        rep.lifting_steps += k;
        const double th0 = now_ms();
        // y mod p^k from the per-step combinations (Horner, high digit first)
        BigInt y, pk = BigInt::from_i64(1);
        for (int64_t i = k - 1; i >= 0; i--) y.mul_add_small(p, comb[i]);
        for (int64_t i = 0; i < k; i++) pk.mul_add_small(p, 0);
        BigInt a, d;
        if (dethost::rational_reconstruct(y, pk, BigInt::from_i64(1).shl(Nbits),
                                          BigInt::from_i64(1).shl(Dbits), a, d)) {
          // s~_n <- lcm(s~_n, d)
          BigInt g = BigInt::gcd(K, d);
          K = BigInt::div_exact(K * d, g);
        }
        t_host += now_ms() - th0;
      }
    }
    rep.sn_bits = K.bit_length();
    rep.t_lif_ms = now_ms() - tl0;

    // ---------------- CRA on det(A)/K with early termination (Alg. 2.1)
    const double tc0 = now_ms();
    const int bits = o.prime_bits;
    const double log2_l = (double)(bits - 1);
    const double log2_HK = std::max(0.0, bd.log2_h - (double)(K.bit_length() - 1));
    const double logl_H = std::max(1.0, log2_HK / log2_l);
    int64_t kET = dethost::et_run_length(o.log2_inv_eps, dethost::prime_set_size(bits), logl_H);
    if (kET < 0) kET = INT64_MAX;                    // lemma not applicable: certify only
    dethost::PrimeSampler samp(dethost::splitmix64(rng), bits);
    dethost::CrtState crt;
    bool done = false;
    int64_t batch = std::min<int64_t>(std::max<int64_t>(kET + 3, 8), 64);
    std::vector<uint32_t> ps, rs;
    while (!done) {
      ps.resize(batch);
      rs.resize(batch);
      for (int64_t i = 0; i < batch; i++) ps[i] = samp.next();
      TRY(residues_core(c, dA, dlda, (int)n, ps.data(), batch, rs.data(), int8));
      rep.et_rounds++;
      const double th0 = now_ms();
      for (int64_t i = 0; i < batch && !done; i++) {
        const uint32_t p = ps[i];
        const uint64_t km = K.mod_small(p);
        if (km == 0) continue;                       // p | K: skip this prime
        const uint64_t kinv = dethost::powmod64(km, p - 2, p);
        const uint32_t d = (uint32_t)dethost::mulmod64(rs[i], kinv, p);
        crt.add(p, d);
        rep.primes_used++;
        // deterministic stop: prod p >= 2 H / K  (log2 M >= 1 + log2 H - log2 K)
        if ((double)(crt.M.bit_length() - 1) >= 1.0 + log2_HK + 1.0) done = true;
        else if (!o.certify && crt.same >= kET) {
          done = true;
          rep.early_terminated = 1;
        }
      }
      t_host += now_ms() - th0;
      if (!done) {
        const double need = (1.0 + log2_HK + 1.0 - (double)(crt.M.bit_length() - 1)) / log2_l;
        batch = std::min<int64_t>(std::max<int64_t>((int64_t)ceil(need) + 1, 4), 512);
        if (!o.certify) batch = std::min<int64_t>(batch, std::max<int64_t>(2 * kET, 8));
      }
    }
    rep.t_cra_ms = now_ms() - tc0;
    const double th1 = now_ms();
    BigInt det = crt.r * K;
    t_host += now_ms() - th1;
    rep.t_host_ms = t_host;
    if (report) *report = rep;
    (void)t0;
    return emit(det);
  } catch (const std::exception& e) {
    return fail(c, DET_E_NOMEM, e.what());
  } catch (...) {
    return fail(c, DET_E_INVALID, "unexpected error");
  }
}

}  // extern "C"
