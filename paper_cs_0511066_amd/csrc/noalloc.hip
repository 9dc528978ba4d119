// det_mod_primes_noalloc: the modular determinants of det_mod_primes (FP64
// trailing updates, single-level blocking) with every device buffer taken from
// one file-scope device array instead of the library's allocator, for callers
// that cannot allocate device memory.  The kernels are those of
// det_mod_primes (residue reduction, panel, fused LU-step update, det
// finalisation); they receive pointers into the array as they receive the
// context's workspace there.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "../../include/det.h"
#include "host_numerics.hpp"
#include "kernels.hpp"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)64 << 20;   // 64 MiB per device
constexpr int MAX_DEVICES = 64;
constexpr int MAX_BATCH = 63;     // below the two-level threshold of det_mod_primes

// The per-device scratch memory.  In host code this name is only a handle for
// hipGetSymbolAddress; kernels receive the address obtained from it.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

// Address of the array on `device` (which must be current), looked up once.
hipError_t scratch_address(int device, unsigned char** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *out = (unsigned char*)g_ptr[device];
  return hipSuccess;
}

struct PrimeArg {
  uint32_t p[MAX_BATCH];
};

// Moduli of a batch (p and its correctly rounded reciprocal, as the host
// computes them) and zeroed singularity flags.
__global__ void k_batch_setup(PrimeArg pa, int count, detk::Modulus* mods, int32_t* flags) {
  const int i = threadIdx.x;
  if (i < count) {
    mods[i].p = (double)pa.p[i];
    mods[i].pinv = 1.0 / (double)pa.p[i];
    flags[i] = 0;
  }
}

// *amax = max |a_ij| over the n x n matrix (as an unsigned 64-bit integer);
// *amax must be zero at launch.
__global__ void k_abs_max(const int64_t* __restrict__ A, int64_t lda, int n,
                          unsigned long long* amax) {
  unsigned long long m = 0;
  for (int i = blockIdx.x; i < n; i += gridDim.x)
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      const int64_t v = A[(int64_t)i * lda + j];
      const unsigned long long u = v < 0 ? 0ull - (unsigned long long)v : (unsigned long long)v;
      m = u > m ? u : m;
    }
  atomicMax(amax, m);
}

__global__ void k_zero_u64(unsigned long long* v) { *v = 0; }

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

struct Layout {
  int64_t ldw, slab, w, piv, flags, mods, linv, res, amax, total;
};

// Offsets of a batch of `nit` items of order n inside the array.
Layout layout(int64_t n, int64_t nit) {
  Layout L;
  L.ldw = (n + 63) / 64 * 64 + 32;                 // as det_mod_primes' workspace rows
  L.slab = L.ldw * n;
  L.amax = 0;
  L.w = 256;
  L.piv = align256(L.w + nit * L.slab * 4);
  L.flags = align256(L.piv + nit * n * 4);
  L.mods = align256(L.flags + nit * 4);
  L.linv = align256(L.mods + nit * (int64_t)sizeof(detk::Modulus));
  L.res = align256(L.linv + nit * 32 * 32 * 4);
  L.total = align256(L.res + nit * 4);
  return L;
}

// Largest K with K h^2 + h <= 2^53, h = (pmax - 1) / 2 (exact FP64 sums).
int exact_chunk(uint32_t pmax) {
  const double h = (double)((pmax - 1) / 2);
  return (int)std::min(floor((9007199254740992.0 - h) / (h * h)), 1e6);
}

}  // namespace

extern "C" det_status det_mod_primes_noalloc(int device, void* hip_stream, const int64_t* A,
                                             int64_t n, int64_t lda, const uint32_t* primes,
                                             int64_t nprimes, uint32_t* residues) {
  if (n < 0 || nprimes < 0 || (nprimes > 0 && (!primes || !residues)) ||
      (n > 0 && (!A || lda < n)) || device < 0 || device >= MAX_DEVICES)
    return DET_E_INVALID;
  for (int64_t i = 0; i < nprimes; i++) {
    const uint32_t q = primes[i];
    if (q < 3 || q >= (1u << 26)) return DET_E_PRIME_RANGE;
    if (!dethost::is_prime_u32(q)) return DET_E_NOT_PRIME;
  }
  if (n == 0 || nprimes == 0) {
    for (int64_t i = 0; i < nprimes; i++) residues[i] = 1 % primes[i];
    return DET_OK;
  }
  if (layout(n, 1).total > (int64_t)SCRATCH_BYTES) return DET_E_INVALID;   // one item must fit
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess || hipSetDevice(device) != hipSuccess) return DET_E_DEVICE;
  struct Restore {
    int d;
    ~Restore() { (void)hipSetDevice(d); }
  } restore{prev};
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, A) != hipSuccess || attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return DET_E_INVALID;                          // A must be device memory
  }
  unsigned char* base = nullptr;
  if (scratch_address(device, &base) != hipSuccess) return DET_E_DEVICE;
  hipStream_t st = (hipStream_t)hip_stream;
  const int nn = (int)n;
  // entry bound |a_ij| < 2^31 (the FP64 residue reduction reads exact values)
  unsigned long long* amax = (unsigned long long*)(base + 0);
  unsigned long long h_amax = 0;
  k_zero_u64<<<1, 1, 0, st>>>(amax);
  k_abs_max<<<std::min(nn, 1024), 256, 0, st>>>(A, lda, nn, amax);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&h_amax, amax, sizeof(h_amax), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return DET_E_DEVICE;
  if (h_amax >= (1ull << 31)) return DET_E_OVERFLOW;

  int64_t bmax = MAX_BATCH;
  while (bmax > 1 && layout(n, bmax).total > (int64_t)SCRATCH_BYTES) bmax--;
  for (int64_t s0 = 0; s0 < nprimes; s0 += bmax) {
    const int nit = (int)std::min<int64_t>(bmax, nprimes - s0);
    const Layout L = layout(n, nit);
    int32_t* W = (int32_t*)(base + L.w);
    int32_t* piv = (int32_t*)(base + L.piv);
    int32_t* flags = (int32_t*)(base + L.flags);
    detk::Modulus* mods = (detk::Modulus*)(base + L.mods);
    int32_t* linv = (int32_t*)(base + L.linv);
    uint32_t* res = (uint32_t*)(base + L.res);
    PrimeArg pa{};
    uint32_t pmax = 0;
    for (int i = 0; i < nit; i++) {
      pa.p[i] = primes[s0 + i];
      pmax = std::max(pmax, pa.p[i]);
    }
    const int kc = exact_chunk(pmax), kc4 = std::max(1, kc / 4);
    k_batch_setup<<<1, 64, 0, st>>>(pa, nit, mods, flags);
    if (hipGetLastError() != hipSuccess) return DET_E_DEVICE;
    if (detk::launch_residues(A, lda, nn, nn, W, L.ldw, L.slab, mods, nit, st) != hipSuccess)
      return DET_E_DEVICE;
    for (int j0 = 0; j0 < nn;) {
      const int pbw = detk::panel_width_for(nn - j0);
      const int pb = std::min(pbw, nn - j0);
      if (detk::launch_panel(W, L.ldw, L.slab, nn, j0, pb, pbw, mods, piv, n, flags, linv,
                             nullptr, kc, nit, nn, st) != hipSuccess)
        return DET_E_DEVICE;
      const int rest = nn - (j0 + pb);
      if (detk::launch_lu_update(W, L.slab, L.ldw, j0, pb, rest, rest, linv, pbw, nullptr, mods,
                                 kc4, nullptr, 0, nit, st) != hipSuccess)
        return DET_E_DEVICE;
      j0 += pb;
    }
    if (detk::launch_det_finalize(W, L.ldw, L.slab, nn, piv, n, flags, mods, res, nit, st) !=
            hipSuccess ||
        hipMemcpyAsync(residues + s0, res, nit * sizeof(uint32_t), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return DET_E_DEVICE;
  }
  return DET_OK;
}
