// Batched exact determinants (det_batch) and the autotuner of the persistent
// LU kernel (det_autotune).
//
// Every matrix of the batch follows the early-terminated Chinese remaindering
// of Section 2.1 (Alg. 2.1 with the run length of Lemma 2.1(iv)), and the
// rounds of all matrices run together: a round draws the next primes of
// every unfinished matrix, puts all (matrix, prime) LU items of orders up to
// the queue kernel's limit into one device work queue sorted by decreasing
// order, and runs them in one persistent launch (captured in a HIP graph
// together with the queue reset and the copies); larger matrices take the
// blocked batched LU of det_mod_primes on the second stream meanwhile.  The
// host then feeds each matrix's residues, in draw order, to its Garner
// reconstruction and stops it as Alg. 2.1 does.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <numeric>
#include <exception>
#include <string>
#include <chrono>
#include <thread>
#include <vector>

#include "../../include/det.h"
#include "bigint.hpp"
#include "cra.hpp"
#include "ctx.hpp"
#include "host_numerics.hpp"
#include "kernels.hpp"

using dethost::BigInt;

constexpr int QUEUE_BUCKETS[] = {64, 128, 256, 512};

// The queue kernel's launch shape for a set of items whose largest order is
// nmax: the autotuned entry of the smallest bucket that holds nmax, else
// panel width 32 with one workgroup per CU.
void queue_shape(const det_ctx* c, int nmax, int* variant, int* grid_per_cu) {
  *variant = detk::LU_QUEUE_PB32;
  *grid_per_cu = 1;
  for (const auto& t : c->tune)
    if (nmax <= t.nmax) {
      *variant = t.variant;
      *grid_per_cu = t.blocks_per_cu;
      return;
    }
}

// Starts `items` through the persistent LU kernel on stream st and returns
// at once: item i's residue appears in q_hout (mapped host memory, 0xFFFFFFFF
// until written) at the item's queue position, which *qpos receives in the
// items' own order (out_index).  With `graph` the copy of the items, the
// queue reset and the launch are captured into a HIP graph and launched as
// one.  queue_wait ends it.
det_status queue_start(det_ctx* c, std::vector<detk::LuItem>& items, std::vector<int32_t>* qpos,
                       hipStream_t st, bool graph, int variant, int grid_per_cu) {
  const int nit = (int)items.size();
  if (nit == 0) return DET_OK;
  int nmax = 0;
  for (const auto& it : items) nmax = std::max(nmax, (int)it.n);
  if (nmax > detk::lu_queue_max_n(variant)) return fail(c, DET_E_INVALID, "order above the queue limit");
  const int grid = std::max(1, std::min(nit, c->cus * grid_per_cu));
  const int64_t ws_stride = detk::lu_queue_ws_stride(nmax);
  const int64_t aux_stride = detk::lu_queue_aux_stride();
  // results are indexed by position in the queue
  int32_t omax = -1;
  for (const auto& it : items) omax = std::max(omax, it.out_index);
  qpos->assign((size_t)omax + 1, -1);
  for (int i = 0; i < nit; i++) {
    (*qpos)[items[i].out_index] = i;
    items[i].out_index = i;
  }
  void* dout = nullptr;
  TRY(ensure(c, c->q_items, (size_t)nit * sizeof(detk::LuItem), st));
  TRY(ensure(c, c->q_next, 256, st));
  TRY(ensure(c, c->q_ws, (size_t)grid * ws_stride * sizeof(int32_t), st));
  TRY(ensure(c, c->q_aux, (size_t)grid * aux_stride * sizeof(int32_t), st));
  TRY(ensure_pin(c, c->q_hitems, (size_t)nit * sizeof(detk::LuItem), st));
  TRY(ensure_mapped(c, c->q_hout, (size_t)nit * sizeof(uint32_t), st, &dout));
  memcpy(c->q_hitems.p, items.data(), (size_t)nit * sizeof(detk::LuItem));
  memset(c->q_hout.p, 0xFF, (size_t)nit * sizeof(uint32_t));
  for (int i = 0; i < nit; i++) items[i].out_index = -1;      // (the caller's order is in qpos)
  auto enqueue = [&]() -> det_status {
    HIPCHK(hipMemcpyAsync(c->q_items.p, c->q_hitems.p, (size_t)nit * sizeof(detk::LuItem),
                          hipMemcpyHostToDevice, st));
    HIPCHK(detk::launch_queue_reset((unsigned*)c->q_next.p, 1, st));
    HIPCHK(detk::launch_lu_queue(variant, grid, (const detk::LuItem*)c->q_items.p, nit,
                                 (unsigned*)c->q_next.p, (int32_t*)c->q_ws.p, ws_stride,
                                 (int32_t*)c->q_aux.p, (uint32_t*)dout, st));
    return DET_OK;
  };
  if (graph) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const det_status s = enqueue();
    const hipError_t e = hipStreamEndCapture(st, &g);
    if (s != DET_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    HIPCHK(e);
    const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(ei);
    // the executable graph lives until the next start (after the caller's
    // wait) or until the context goes
    if (c->q_exec) (void)hipGraphExecDestroy(c->q_exec);
    c->q_exec = ge;
    HIPCHK(hipGraphLaunch(ge, st));
  } else {
    TRY(enqueue());
  }
  return DET_OK;
}

// Residue of the item at queue position q, or 0xFFFFFFFF while it runs.
uint32_t queue_result(const det_ctx* c, int32_t q) {
  return __atomic_load_n((const uint32_t*)c->q_hout.p + q, __ATOMIC_ACQUIRE);
}

// Blocking form: start, wait, and copy every residue to out_host[out_index].
det_status run_queue(det_ctx* c, std::vector<detk::LuItem>& items, uint32_t* out_host,
                     hipStream_t st, bool graph, int variant, int grid_per_cu) {
  std::vector<int32_t> orig(items.size());
  for (size_t i = 0; i < items.size(); i++) orig[i] = items[i].out_index;
  std::vector<int32_t> qpos;
  TRY(queue_start(c, items, &qpos, st, graph, variant, grid_per_cu));
  HIPCHK(hipStreamSynchronize(st));
  for (size_t i = 0; i < items.size(); i++) {
    items[i].out_index = orig[i];
    if (!items.empty()) out_host[orig[i]] = queue_result(c, qpos[orig[i]]);
  }
  return DET_OK;
}

namespace {

bool graphs_enabled() {
  const char* g = getenv("DET_BATCH_GRAPH");
  return !(g && strcmp(g, "0") == 0);
}

// One matrix of a batch: its staged copy and its Chinese remaindering.
struct Mat {
  const int64_t* dA = nullptr;
  int64_t dlda = 0;
  int n = 0;
  dethost::Bounds bd;
  dethost::CraJob job;
  bool done = false;
};

// ---- the autotuner's cache file: one line a bucket after a header line
bool load_tune(det_ctx* c, const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char arch[64] = {0};
  int cus = 0;
  std::vector<det_ctx::Tune> t;
  bool ok = fscanf(f, " {\"arch\": \"%63[^\"]\", \"cus\": %d, \"buckets\": [", arch, &cus) == 2;
  while (ok) {
    det_ctx::Tune e{};
    if (fscanf(f, " {\"nmax\": %d, \"variant\": %d, \"blocks_per_cu\": %d, \"items_per_ms\": %lf}",
               &e.nmax, &e.variant, &e.blocks_per_cu, &e.items_per_ms) != 4)
      break;
    t.push_back(e);
    if (fscanf(f, " ,") != 0) break;
  }
  fclose(f);
  if (!ok || t.empty() || cus != c->cus || strcmp(arch, c->arch) != 0) return false;
  for (const auto& e : t)
    if (detk::lu_queue_max_n(e.variant) == 0 ||
        e.blocks_per_cu != detk::lu_queue_blocks_per_cu(e.variant))
      return false;
  c->tune = t;
  return true;
}

void save_tune(const det_ctx* c, const char* path) {
  FILE* f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\"arch\": \"%s\", \"cus\": %d, \"buckets\": [\n", c->arch, c->cus);
  for (size_t i = 0; i < c->tune.size(); i++) {
    const auto& e = c->tune[i];
    fprintf(f, "  {\"nmax\": %d, \"variant\": %d, \"blocks_per_cu\": %d, \"items_per_ms\": %.3f}%s\n",
            e.nmax, e.variant, e.blocks_per_cu, e.items_per_ms, i + 1 < c->tune.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  fclose(f);
}

// Times every launch shape of the queue kernel on items of order `nmax`
// (a seeded dense matrix, 23-bit primes, 4 items per CU) and keeps the
// fastest.  Returns its items per ms.
det_status tune_bucket(det_ctx* c, int nmax, det_ctx::Tune* best) {
  hipStream_t st = c->st;
  const int64_t n = nmax;
  std::vector<int64_t> A((size_t)n * n);
  uint64_t s = 0x7475AE + (uint64_t)nmax;
  for (auto& v : A) v = (int64_t)(dethost::splitmix64(s) % 255) - 127;
  TRY(ensure(c, c->Adev, (size_t)n * n * sizeof(int64_t), st));
  HIPCHK(hipMemcpy(c->Adev.p, A.data(), A.size() * sizeof(int64_t), hipMemcpyHostToDevice));
  const int nit = 4 * c->cus;
  dethost::PrimeSampler samp(0x5EED + nmax, 23);
  std::vector<detk::LuItem> items(nit);
  for (int i = 0; i < nit; i++)
    items[i] = detk::LuItem{(const int64_t*)c->Adev.p, n, (int32_t)n, samp.next(), i, 0};
  std::vector<uint32_t> out(nit), ref;
  struct Cand {
    int variant, bpc;
  };
  const Cand cands[] = {{detk::LU_QUEUE_PB32, 1}, {detk::LU_QUEUE_PB16, 1},
                        {detk::LU_QUEUE_PB16X2, 2}};
  best->items_per_ms = -1;
  for (const Cand& cd : cands) {
    TRY(run_queue(c, items, out.data(), st, false, cd.variant, cd.bpc));      // warm-up
    if (ref.empty()) ref = out;
    else if (out != ref) return fail(c, DET_E_DEVICE, "autotune: launch shapes disagree");
    double tmin = 1e30;
    for (int r = 0; r < 2; r++) {
      const double t0 = now_ms();
      TRY(run_queue(c, items, out.data(), st, false, cd.variant, cd.bpc));
      tmin = std::min(tmin, now_ms() - t0);
    }
    const double rate = nit / std::max(tmin, 1e-6);
    if (rate > best->items_per_ms) *best = det_ctx::Tune{nmax, cd.variant, cd.bpc, rate};
  }
  return DET_OK;
}

det_status autotune(det_ctx* c, const char* path) {
  if (path && load_tune(c, path)) return DET_OK;
  std::vector<det_ctx::Tune> t;
  for (int nmax : QUEUE_BUCKETS) {
    det_ctx::Tune b{};
    TRY(tune_bucket(c, nmax, &b));
    t.push_back(b);
  }
  c->tune = t;
  if (path) save_tune(c, path);
  return DET_OK;
}

}  // namespace

extern "C" {

det_status det_autotune(det_ctx* c, const char* cache_path) {
  if (!c) return DET_E_INVALID;
  try {
    HIPCHK(hipSetDevice(c->device));
    return autotune(c, cache_path);
  } catch (const std::exception& e) {
    return fail(c, DET_E_NOMEM, e.what());
  }
}

det_status det_autotune_read(const det_ctx* c, int64_t cap, int32_t* nmax, int32_t* variant,
                             int32_t* blocks_per_cu, double* items_per_ms, int64_t* count) {
  if (!c || !count || cap < 0) return DET_E_INVALID;
  *count = (int64_t)c->tune.size();
  for (int64_t i = 0; i < std::min<int64_t>(cap, *count); i++) {
    if (nmax) nmax[i] = c->tune[i].nmax;
    if (variant) variant[i] = c->tune[i].variant;
    if (blocks_per_cu) blocks_per_cu[i] = c->tune[i].blocks_per_cu;
    if (items_per_ms) items_per_ms[i] = c->tune[i].items_per_ms;
  }
  return DET_OK;
}

det_status det_batch(det_ctx* c, int64_t count, const int64_t* const* A, const int64_t* n,
                     const int64_t* lda, const det_opts* opts_in, int* sign, uint32_t* mag,
                     int64_t limb_stride, int64_t* limb_count, det_status* status,
                     double* t_done_ms) {
  if (!c) return DET_E_INVALID;
  const double t0 = now_ms();
  try {
    if (count < 0 || limb_stride < 0 || (limb_stride > 0 && count > 0 && !mag))
      return fail(c, DET_E_INVALID, "invalid argument");
    if (count == 0) return DET_OK;
    if (!A || !n || !lda || !sign || !limb_count || !status)
      return fail(c, DET_E_INVALID, "invalid argument");
    det_opts o;
    det_opts_default(&o);
    if (opts_in) o = *opts_in;
    if (!(o.log2_inv_eps > 0)) o.log2_inv_eps = 64.0;
    if (o.prime_bits < 12 || o.prime_bits > 26)
      return fail(c, DET_E_PRIME_RANGE, "prime_bits out of range");
    for (int64_t i = 0; i < count; i++) {
      status[i] = DET_OK;
      if (n[i] < 0 || n[i] > 4096 || (n[i] > 0 && (!A[i] || lda[i] < n[i])))
        return fail(c, DET_E_INVALID, "invalid matrix " + std::to_string(i));
    }
    HIPCHK(hipSetDevice(c->device));
    if (c->tune.empty()) TRY(autotune(c, getenv("DET_AUTOTUNE_CACHE")));
    hipStream_t st = c->st;
    // ---- stage the matrices: device pointers in place, host matrices
    // packed into one device buffer (one copy each), all entries |a| < 2^31
    std::vector<Mat> M(count);
    std::vector<char> on_dev(count);
    size_t host_elems = 0;
    for (int64_t i = 0; i < count; i++) {
      on_dev[i] = n[i] > 0 && is_device_ptr(A[i]);
      if (!on_dev[i]) host_elems += (size_t)n[i] * n[i];
    }
    TRY(ensure(c, c->q_mats, std::max<size_t>(host_elems, 1) * sizeof(int64_t), st));
    size_t off = 0;
    size_t dev_norms = 0;
    for (int64_t i = 0; i < count; i++) {
      Mat& m = M[i];
      m.n = (int)n[i];
      if (m.n == 0) continue;
      if (on_dev[i]) {
        m.dA = A[i];
        m.dlda = lda[i];
        dev_norms += 3 * (size_t)m.n;
        continue;
      }
      for (int64_t r = 0; r < n[i]; r++)
        for (int64_t j = 0; j < n[i]; j++) {
          const int64_t v = A[i][r * lda[i] + j];
          if (v >= (1LL << 31) || v <= -(1LL << 31))
            return fail(c, DET_E_OVERFLOW, "matrix entry with |a_ij| >= 2^31");
        }
      int64_t* dst = (int64_t*)c->q_mats.p + off;
      HIPCHK(hipMemcpy2DAsync(dst, n[i] * sizeof(int64_t), A[i], lda[i] * sizeof(int64_t),
                              n[i] * sizeof(int64_t), n[i], hipMemcpyHostToDevice, st));
      m.dA = dst;
      m.dlda = n[i];
      m.bd = dethost::bounds_host(A[i], n[i], lda[i]);
      off += (size_t)n[i] * n[i];
    }
    if (dev_norms) {
      // bounds of device matrices: the norm kernels of every matrix, one wait
      TRY(ensure(c, c->norms, dev_norms * sizeof(double), st));
      size_t o2 = 0;
      for (int64_t i = 0; i < count; i++)
        if (on_dev[i]) {
          double* nb = (double*)c->norms.p + o2;
          HIPCHK(detk::launch_norms(M[i].dA, M[i].dlda, M[i].n, nb, nb + 2 * M[i].n, st));
          o2 += 3 * (size_t)M[i].n;
        }
      std::vector<double> h(dev_norms);
      HIPCHK(hipMemcpyAsync(h.data(), c->norms.p, dev_norms * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      o2 = 0;
      for (int64_t i = 0; i < count; i++)
        if (on_dev[i]) {
          const int nn = M[i].n;
          const double* nb = h.data() + o2;
          double amax = 0;
          for (int j = 0; j < nn; j++) amax = std::max(amax, nb[2 * nn + j]);
          if (amax >= 2147483648.0) return fail(c, DET_E_OVERFLOW, "matrix entry with |a_ij| >= 2^31");
          std::vector<double> cols(nb, nb + nn), rows(nb + nn, nb + 2 * nn);
          M[i].bd = dethost::bounds_from_sums(cols, rows, amax);
          o2 += 3 * (size_t)nn;
        }
    } else {
      HIPCHK(hipStreamSynchronize(st));
    }
    // ---- per-matrix Chinese remaindering set-up (Alg. 2.1, Lemma 2.1(iv))
    const int bits = o.prime_bits;
    int64_t left = 0;
    auto emit = [&](int64_t i, const BigInt& v) {
      std::vector<uint32_t> l = v.limbs32();
      sign[i] = v.sign;
      limb_count[i] = (int64_t)l.size();
      if ((int64_t)l.size() > limb_stride) status[i] = DET_E_BUFFER_TOO_SMALL;
      else if (!l.empty()) memcpy(mag + i * limb_stride, l.data(), l.size() * sizeof(uint32_t));
      if (t_done_ms) t_done_ms[i] = now_ms() - t0;
    };
    for (int64_t i = 0; i < count; i++) {
      Mat& m = M[i];
      if (m.n == 0) {
        emit(i, BigInt::from_i64(1));
        m.done = true;
        continue;
      }
      m.job.init(m.bd, m.n, o.seed + (uint64_t)i, bits, o.log2_inv_eps, o.certify != 0);
      left++;
    }
    // ---- rounds
    const bool graph = graphs_enabled();
    const int qmax = detk::lu_queue_max_n(detk::LU_QUEUE_PB32);
    std::vector<uint32_t> res;
    for (int round = 0; left > 0; round++) {
      std::vector<detk::LuItem> items;
      std::vector<int64_t> big;                  // matrices above the queue limit
      int64_t nres = 0;
      for (int64_t i = 0; i < count; i++) {
        Mat& m = M[i];
        if (m.done) continue;
        const int64_t want = m.job.next_count();
        m.job.draw(want, nres);
        nres += want;
        if (m.n > qmax) {
          big.push_back(i);
          continue;
        }
        for (int64_t k = 0; k < want; k++)
          items.push_back(detk::LuItem{m.dA, m.dlda, m.n, m.job.ps[k], (int32_t)(m.job.res0 + k), 0});
      }
      res.assign(nres, 0);
      // smallest orders first: their matrices complete early, and with many
      // items per order the queue still balances the workgroups
      std::stable_sort(items.begin(), items.end(),
                       [](const detk::LuItem& a, const detk::LuItem& b) { return a.n < b.n; });
      int nmax = 0;
      for (const auto& it : items) nmax = std::max(nmax, (int)it.n);
      int variant, bpc;
      queue_shape(c, nmax, &variant, &bpc);
      // big matrices on the second stream while the queue runs on st
      det_status big_st = DET_OK;
      std::thread big_thread;
      if (!big.empty()) {
        HIPCHK(hipEventRecord(c->ev, st));       // the staged matrices are on st
        HIPCHK(hipStreamWaitEvent(c->own2, c->ev, 0));
        big_thread = std::thread([&] {
          (void)hipSetDevice(c->device);
          for (int64_t i : big) {
            Mat& m = M[i];
            const det_status s = drv_residues(c, c->ws[1], m.dA, m.dlda, m.n, m.job.ps.data(),
                                              (int64_t)m.job.ps.size(), res.data() + m.job.res0,
                                              o.path);
            if (s != DET_OK) {
              big_st = s;
              return;
            }
          }
        });
      }
      std::vector<int32_t> qpos;
      det_status qs = queue_start(c, items, &qpos, st, graph, variant, bpc);
      // ---- host: as soon as all residues of a matrix of this round are in,
      // its Garner steps in draw order with Alg. 2.1's stop, while the queue
      // keeps running
      auto finish = [&](int64_t i) {
        Mat& m = M[i];
        if (m.job.absorb(res.data())) {
          m.done = true;
          emit(i, m.job.crt.r);
          left--;
        }
      };
      std::vector<int64_t> pend;
      for (int64_t i = 0; i < count; i++)
        if (!M[i].done && !M[i].job.ps.empty() && M[i].n <= qmax) pend.push_back(i);
      while (qs == DET_OK && !pend.empty()) {
        size_t keep = 0;
        for (size_t u = 0; u < pend.size(); u++) {
          Mat& m = M[pend[u]];
          bool all = true;
          for (size_t k = 0; k < m.job.ps.size() && all; k++) {
            const uint32_t v = queue_result(c, qpos[m.job.res0 + k]);
            if (v == 0xFFFFFFFFu) all = false;
            else res[m.job.res0 + k] = v;
          }
          if (all) finish(pend[u]);
          else pend[keep++] = pend[u];
        }
        pend.resize(keep);
        if (!pend.empty()) {
          // a stalled device (error) would never fill the slots: check it
          const hipError_t q = hipStreamQuery(st);
          if (q != hipSuccess && q != hipErrorNotReady) qs = fail(c, DET_E_DEVICE, hipGetErrorString(q));
          else if (q == hipSuccess) {
            // the queue is done: every slot is written
            for (int64_t i : pend) {
              Mat& m = M[i];
              for (size_t k = 0; k < m.job.ps.size(); k++)
                res[m.job.res0 + k] = queue_result(c, qpos[m.job.res0 + k]);
              finish(i);
            }
            pend.clear();
          } else {
            std::this_thread::sleep_for(std::chrono::microseconds(20));
          }
        }
      }
      if (qs == DET_OK) {
        const hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) qs = fail(c, DET_E_DEVICE, hipGetErrorString(e));
      }
      if (big_thread.joinable()) big_thread.join();
      TRY(qs);
      TRY(big_st);
      for (int64_t i : big) finish(i);
    }
    for (int64_t i = 0; i < count; i++)
      if (status[i] != DET_OK)
        return fail(c, status[i], "matrix " + std::to_string(i) + ": " + det_status_str(status[i]));
    return DET_OK;
  } catch (const std::exception& e) {
    return fail(c, DET_E_NOMEM, e.what());
  } catch (...) {
    return fail(c, DET_E_INVALID, "unexpected error");
  }
}

}  // extern "C"
