// Internal state shared by the C-ABI sources: the context (det_ctx), its
// device and pinned host buffers, error reporting and kernel timing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/det.h"
#include "kernels.hpp"

// A grow-only device buffer of the context.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
};

inline double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Pinned host memory for the small transfers of the path: an asynchronous
// copy from pageable memory can hold the host until earlier work drains,
// which would serialize the two streams of a context.
struct PinBuf {
  void* p = nullptr;
  size_t cap = 0;
};

// Device workspace of one batched LU, bound to one stream.
struct LuWs {
  DevBuf W, piv, flags, mods, linv, uinv, tinv, limbA, limbB, res, cnt;
  PinBuf hmods;                 // pinned host copy of the moduli (async uploads)
  PinBuf hflags;                // pinned copy of the batch's flags (block-pivot check)
  hipStream_t st = nullptr;
};

struct det_ctx {
  int device = 0;
  size_t budget = 0;
  size_t held = 0;
  hipStream_t own = nullptr;     // the context's stream (default for ws[0])
  hipStream_t own2 = nullptr;    // second stream: CRA batches beside the Dixon solve
  hipStream_t st = nullptr;      // current stream of ws[0] (own or the caller's)
  hipEvent_t ev = nullptr;       // orders own2 after work queued on st
  hipEvent_t ev_cra = nullptr;   // the same for the first CRA batch (enqueued by a second thread)
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;   // device time of the first CRA batch
  hipEvent_t ev_det = nullptr;   // det(A) mod the lifting primes read back (from the inverse's LU)
  std::mutex mu;                 // the error text, the budget count, the kernel timing state
  std::string err;
  LuWs ws[2];
  DevBuf Adev, norms, Cu, Ai, r, rp, x, digits, comb, cvec, sync, C1, E, rp1, x1, C2, Ed,
      rv, xv, Hp;
  uint32_t* hres = nullptr;      // pinned host residues of the background batch
  size_t hres_cap = 0;
  PinBuf hstage;                 // pinned staging of the lifting's vectors and results
  PinBuf hsmall;                 // pinned flags and error words read back on st
  PinBuf hnorms;                 // pinned read-back of the column and row norms
  PinBuf hcomb;                  // pinned read-back of the combination sums of the liftings
  int lift_mode = 0;             // 0: fastest cooperative form that applies; 1: one launch per
                                 // phase; 2: the 64-bit integer form modulo p^2
  bool block_pivots = true;      // the inverse's panels search their diagonal block first
  bool hensel_i8 = true;         // Hensel planes on int8 MFMA where the operands allow it
  int64_t block_pivot_retries = 0;   // inverses that fell back to the full pivot search
  // kernel timing (det_profile_select / det_profile_read)
  int prof_kind = 0;
  int64_t prof_launches = 0;
  double prof_bytes = 0, prof_ops = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending;
  std::vector<hipEvent_t> ev_pool;
  // the persistent LU over a work queue (det_batch, the serving loop): item
  // array, queue counters, per-workgroup slabs and pivot records, residues,
  // and their pinned host copies
  DevBuf q_items, q_next, q_ws, q_aux, q_out, q_mats;
  PinBuf q_hitems, q_hout;
  hipGraphExec_t q_exec = nullptr;   // the last round's executable graph
  // autotuned launch shape of the queue kernel per order bucket (det_autotune)
  struct Tune {
    int nmax, variant, blocks_per_cu;
    double items_per_ms;
  };
  std::vector<Tune> tune;
  int cus = 0;                   // compute units of the device
  char arch[64] = {0};           // its gcnArchName
};

inline det_status fail(det_ctx* c, det_status s, const std::string& msg) {
  if (c) {
    std::lock_guard<std::mutex> lk(c->mu);
    c->err = msg;
  }
  return s;
}

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(c, DET_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TRY(expr)                     \
  do {                                \
    det_status s_ = (expr);           \
    if (s_ != DET_OK) return s_;      \
  } while (0)

// Grow-only device buffer used on stream `st`; the previous contents are not kept.
inline det_status ensure(det_ctx* c, DevBuf& b, size_t bytes, hipStream_t st) {
  if (bytes == 0) bytes = 16;
  if (b.cap >= bytes) return DET_OK;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->budget && c->held - b.cap + bytes > c->budget) {
      c->err = "device workspace would exceed the context's HBM budget";
      return DET_E_NOMEM;
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  if (b.p) {
    HIPCHK(hipFree(b.p));
    {
      std::lock_guard<std::mutex> lk(c->mu);
      c->held -= b.cap;
    }
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
  std::lock_guard<std::mutex> lk(c->mu);
  c->held += bytes;
  return DET_OK;
}

inline det_status ensure(det_ctx* c, DevBuf& b, size_t bytes) { return ensure(c, b, bytes, c->st); }

// Grow a pinned host buffer that kernels may write directly (mapped, coherent:
// device stores reach host memory without a copy); dev receives its device
// address.  `st` is the stream whose work may still use it.
inline det_status ensure_mapped(det_ctx* c, PinBuf& b, size_t bytes, hipStream_t st, void** dev) {
  if (b.cap < bytes) {
    if (b.p) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(hipHostFree(b.p));
      b.p = nullptr;
      b.cap = 0;
    }
    const size_t cap = std::max<size_t>(bytes, 4096);
    if (hipHostMalloc(&b.p, cap, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      (void)hipGetLastError();
      b.p = nullptr;
      return fail(c, DET_E_NOMEM, "hipHostMalloc (mapped) failed");
    }
    b.cap = cap;
  }
  HIPCHK(hipHostGetDevicePointer(dev, b.p, 0));
  return DET_OK;
}

// Grow a pinned host buffer; `st` is the stream whose copies may still read it.
inline det_status ensure_pin(det_ctx* c, PinBuf& b, size_t bytes, hipStream_t st) {
  if (b.cap >= bytes) return DET_OK;
  if (b.p) {
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipHostFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  const size_t cap = std::max<size_t>(bytes, 4096);
  if (hipHostMalloc(&b.p, cap, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(c, DET_E_NOMEM, "hipHostMalloc failed");
  }
  b.cap = cap;
  return DET_OK;
}

// Brackets one launch with HIP events on its stream when its kernel class is
// the selected one; the counts are the launcher's algorithmic bytes and ops.
struct ProfScope {
  det_ctx* c;
  hipStream_t st;
  hipEvent_t e1 = nullptr;
  ProfScope(det_ctx* ctx, int kind, double bytes, double ops, hipStream_t stream)
      : c(ctx), st(stream) {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->prof_kind != kind) return;
    hipEvent_t e0 = take(), e = take();
    if (!e0 || !e) return;
    if (hipEventRecord(e0, st) != hipSuccess) return;
    e1 = e;
    c->prof_pending.push_back({e0, e1});
    c->prof_launches++;
    c->prof_bytes += bytes;
    c->prof_ops += ops;
  }
  ~ProfScope() {
    if (e1) (void)hipEventRecord(e1, st);
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

inline bool is_device_ptr(const void* p) {
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice;
}

// Driver steps defined in capi.cpp: the modular determinants of a staged
// device matrix for a list of primes on workspace w (synchronous), and the
// range and primality check of a prime list.
det_status drv_residues(det_ctx* c, LuWs& w, const int64_t* dA, int64_t dlda, int n,
                        const uint32_t* primes, int64_t np, uint32_t* out, det_path path);
det_status drv_check_primes(det_ctx* c, const uint32_t* primes, int64_t np, uint32_t limit);

// The persistent LU queue (batch.cpp): its autotuned launch shape for items
// of orders up to nmax; starting a set of items on stream st (each residue
// then appears in mapped host memory at the item's queue position, which
// qpos maps from the items' out_index); and reading one residue (0xFFFFFFFF
// while it runs).
void queue_shape(const det_ctx* c, int nmax, int* variant, int* grid_per_cu);
det_status queue_start(det_ctx* c, std::vector<detk::LuItem>& items, std::vector<int32_t>* qpos,
                       hipStream_t st, bool graph, int variant, int grid_per_cu);
uint32_t queue_result(const det_ctx* c, int32_t q);
