// The serving loop (det_server_*): a stream of determinant requests, admitted
// by their HBM footprint and served with continuous batching on one context.
//
// One engine thread owns the context.  Each turn it admits waiting requests
// in arrival order while their resident footprint (the matrix copied into
// HBM) fits the budget, then runs one round of the Chinese-remaindering loop
// (Section 2.1, Alg. 2.1) for every admitted request of order <= 512: all
// their (matrix, prime) LU items go into one persistent launch over the
// device work queue, and each request takes its residues, in draw order, as
// soon as they arrive in mapped host memory; a request that early-terminates
// (or reaches the Hadamard bound) completes there and frees its memory for
// the next admission.  Requests that arrive meanwhile join the next round.
// Requests of larger order follow Section 4's introspective scheme (one Dixon
// solve for a large divisor s~_n of det, then the CRA loop on det / s~_n):
// one such request runs between two rounds, with the whole device.
#include <hip/hip_runtime.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <exception>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/det.h"
#include "bigint.hpp"
#include "cra.hpp"
#include "ctx.hpp"
#include "host_numerics.hpp"
#include "kernels.hpp"

using dethost::BigInt;

namespace {

constexpr int QUEUE_MAX_N = 512;

struct Request {
  int64_t id = 0;
  int n = 0;
  std::vector<int64_t> A;          // host copy (row-major n x n), until admitted
  DevBuf dA;                       // the resident copy while admitted
  size_t footprint = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int state = 0;                   // 0 waiting, 1 admitted, 2 done
  det_status status = DET_OK;
  dethost::Bounds bd;
  dethost::CraJob job;
  int sign = 0;
  std::vector<uint32_t> mag;
};

}  // namespace

struct det_server {
  det_ctx* c = nullptr;
  det_opts o;
  size_t budget = 0;
  size_t used = 0, peak = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> waiting;
  std::vector<Request*> admitted;
  std::unordered_map<int64_t, std::unique_ptr<Request>> all;
  int64_t next_id = 0;
  bool stop = false;
  std::thread engine;
  // statistics
  int64_t rounds = 0, completed = 0, max_admitted = 0, queue_items = 0;
};

namespace {

size_t footprint_of(int n) { return (size_t)n * n * sizeof(int64_t) + 4096; }

// The result of a finished request, stored for det_server_poll.
void complete(det_server* s, Request* r, const BigInt& v, det_status st) {
  std::lock_guard<std::mutex> lk(s->mu);
  r->status = st;
  if (st == DET_OK) {
    r->sign = v.sign;
    r->mag = v.limbs32();
  }
  r->t_done = now_ms();
  r->state = 2;
  s->used -= r->footprint;
  s->completed++;
  s->cv_done.notify_all();
}

void release(det_server* s, Request* r) {
  if (r->dA.p) (void)hipFree(r->dA.p);
  r->dA.p = nullptr;
  r->dA.cap = 0;
  std::vector<int64_t>().swap(r->A);
}

// Admission in arrival order while the resident footprint fits the budget
// (a request larger than the whole budget is admitted alone).  Copies each
// admitted matrix into HBM and sets up its reconstruction.
det_status admit(det_server* s) {
  std::vector<Request*> now;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->waiting.empty()) {
      Request* r = s->waiting.front();
      const bool alone = s->admitted.empty() && now.empty();
      if (s->used + r->footprint > s->budget && !alone) break;
      s->waiting.pop_front();
      s->used += r->footprint;
      s->peak = std::max(s->peak, s->used);
      now.push_back(r);
    }
  }
  det_ctx* c = s->c;
  for (Request* r : now) {
    r->t_admit = now_ms();
    const size_t bytes = std::max<size_t>((size_t)r->n * r->n * sizeof(int64_t), 16);
    if (hipMalloc(&r->dA.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      r->dA.p = nullptr;
      complete(s, r, BigInt(), DET_E_NOMEM);
      continue;
    }
    r->dA.cap = bytes;
    if (r->n > 0)
      HIPCHK(hipMemcpyAsync(r->dA.p, r->A.data(), (size_t)r->n * r->n * sizeof(int64_t),
                            hipMemcpyHostToDevice, c->st));
    r->bd = dethost::bounds_host(r->A.data(), r->n, r->n);
    r->job.init(r->bd, r->n, s->o.seed + (uint64_t)r->id, s->o.prime_bits, s->o.log2_inv_eps,
                s->o.certify != 0);
    r->state = 1;
    std::lock_guard<std::mutex> lk(s->mu);
    s->admitted.push_back(r);
    s->max_admitted = std::max<int64_t>(s->max_admitted, (int64_t)s->admitted.size());
  }
  HIPCHK(hipStreamSynchronize(c->st));
  return DET_OK;
}

// One round of the CRA loop for every admitted request of order <= 512.
det_status cra_round(det_server* s) {
  det_ctx* c = s->c;
  std::vector<Request*> reqs;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Request* r : s->admitted)
      if (r->state == 1 && r->n > 0 && r->n <= QUEUE_MAX_N) reqs.push_back(r);
  }
  if (reqs.empty()) return DET_OK;
  std::vector<detk::LuItem> items;
  int64_t nres = 0;
  for (Request* r : reqs) {
    const int64_t want = r->job.next_count();
    r->job.draw(want, nres);
    nres += want;
    for (int64_t k = 0; k < want; k++)
      items.push_back(detk::LuItem{(const int64_t*)r->dA.p, r->n, r->n, r->job.ps[k],
                                   (int32_t)(r->job.res0 + k), 0});
  }
  std::stable_sort(items.begin(), items.end(),
                   [](const detk::LuItem& a, const detk::LuItem& b) { return a.n < b.n; });
  int nmax = 0;
  for (const auto& it : items) nmax = std::max(nmax, (int)it.n);
  int variant, bpc;
  queue_shape(c, nmax, &variant, &bpc);
  std::vector<uint32_t> res(nres, 0);
  std::vector<int32_t> qpos;
  s->queue_items += (int64_t)items.size();
  TRY(queue_start(c, items, &qpos, c->st, true, variant, bpc));
  std::vector<Request*> pend(reqs);
  det_status qs = DET_OK;
  while (!pend.empty()) {
    size_t keep = 0;
    for (Request* r : pend) {
      bool all = true;
      for (size_t k = 0; k < r->job.ps.size() && all; k++) {
        const uint32_t v = queue_result(c, qpos[r->job.res0 + k]);
        if (v == 0xFFFFFFFFu) all = false;
        else res[r->job.res0 + k] = v;
      }
      if (!all) {
        pend[keep++] = r;
        continue;
      }
      if (r->job.absorb(res.data())) complete(s, r, r->job.crt.r, DET_OK);
    }
    pend.resize(keep);
    if (pend.empty()) break;
    const hipError_t q = hipStreamQuery(c->st);
    if (q != hipSuccess && q != hipErrorNotReady) {
      qs = fail(c, DET_E_DEVICE, hipGetErrorString(q));
      break;
    }
    if (q == hipErrorNotReady) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  const hipError_t e = hipStreamSynchronize(c->st);
  if (qs == DET_OK && e != hipSuccess) qs = fail(c, DET_E_DEVICE, hipGetErrorString(e));
  return qs;
}

// The oldest admitted request of order > 512, by the introspective scheme.
det_status solve_one(det_server* s) {
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Request* q : s->admitted)
      if (q->state == 1 && (q->n == 0 || q->n > QUEUE_MAX_N)) {
        r = q;
        break;
      }
  }
  if (!r) return DET_OK;
  if (r->n == 0) {
    complete(s, r, BigInt::from_i64(1), DET_OK);
    return DET_OK;
  }
  det_opts o = s->o;
  o.seed = s->o.seed + (uint64_t)r->id;
  const int64_t cap = 2 * (int64_t)r->n + 16;
  std::vector<uint32_t> mag(cap);
  int sign = 0;
  int64_t cnt = 0;
  det_status st = det_introspective(s->c, (const int64_t*)r->dA.p, r->n, r->n, &o, &sign,
                                    mag.data(), cap, &cnt, nullptr);
  BigInt v;
  if (st == DET_OK) v = BigInt::from_limbs32(mag.data(), (size_t)cnt, sign);
  complete(s, r, v, st);
  return DET_OK;
}

void engine_loop(det_server* s) {
  (void)hipSetDevice(s->c->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        bool active = false;
        for (Request* r : s->admitted) active |= r->state == 1;
        return s->stop || !s->waiting.empty() || active;
      });
      bool active = false;
      for (Request* r : s->admitted) active |= r->state == 1;
      if (s->stop && s->waiting.empty() && !active) return;
    }
    det_status st = admit(s);
    if (st == DET_OK) st = cra_round(s);
    if (st == DET_OK) st = solve_one(s);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->rounds++;
      // finished requests leave the admitted set and free their HBM copy
      std::vector<Request*> keep;
      for (Request* r : s->admitted)
        if (r->state == 2) release(s, r);
        else keep.push_back(r);
      s->admitted.swap(keep);
      if (st != DET_OK) {
        // a device failure ends every request in flight with its status
        for (Request* r : s->admitted) {
          r->status = st;
          r->state = 2;
          r->t_done = now_ms();
          s->used -= r->footprint;
          release(s, r);
        }
        s->admitted.clear();
      }
      s->cv_done.notify_all();
    }
  }
}

}  // namespace

extern "C" {

det_status det_server_create(det_ctx* c, size_t hbm_budget_bytes, const det_opts* opts,
                             det_server** out) {
  if (!c || !out) return DET_E_INVALID;
  *out = nullptr;
  try {
    det_server* s = new det_server();
    s->c = c;
    det_opts_default(&s->o);
    if (opts) s->o = *opts;
    if (!(s->o.log2_inv_eps > 0)) s->o.log2_inv_eps = 64.0;
    if (s->o.prime_bits < 12 || s->o.prime_bits > 26) {
      delete s;
      return fail(c, DET_E_PRIME_RANGE, "prime_bits out of range");
    }
    s->budget = hbm_budget_bytes ? hbm_budget_bytes : ((size_t)16 << 30);
    if (hipSetDevice(c->device) != hipSuccess) {
      delete s;
      return fail(c, DET_E_DEVICE, "hipSetDevice failed");
    }
    if (c->tune.empty()) {
      const det_status st = det_autotune(c, getenv("DET_AUTOTUNE_CACHE"));
      if (st != DET_OK) {
        delete s;
        return st;
      }
    }
    s->engine = std::thread(engine_loop, s);
    *out = s;
    return DET_OK;
  } catch (const std::exception& e) {
    return fail(c, DET_E_NOMEM, e.what());
  }
}

det_status det_server_submit(det_server* s, const int64_t* A, int64_t n, int64_t lda,
                             int64_t* request_id) {
  if (!s || !request_id || n < 0 || n > 4096 || (n > 0 && (!A || lda < n)))
    return DET_E_INVALID;
  try {
    std::unique_ptr<Request> r(new Request());
    r->n = (int)n;
    r->A.resize((size_t)n * n);
    if (n > 0) {
      if (is_device_ptr(A)) {
        if (hipMemcpy2D(r->A.data(), n * sizeof(int64_t), A, lda * sizeof(int64_t),
                        n * sizeof(int64_t), n, hipMemcpyDeviceToHost) != hipSuccess)
          return DET_E_DEVICE;
      } else {
        for (int64_t i = 0; i < n; i++) memcpy(&r->A[i * n], A + i * lda, n * sizeof(int64_t));
      }
      for (int64_t v : r->A)
        if (v >= (1LL << 31) || v <= -(1LL << 31)) return DET_E_OVERFLOW;
    }
    r->footprint = footprint_of((int)n);
    r->t_submit = now_ms();
    std::lock_guard<std::mutex> lk(s->mu);
    r->id = s->next_id++;
    *request_id = r->id;
    s->waiting.push_back(r.get());
    s->all[r->id] = std::move(r);
    s->cv_work.notify_all();
    return DET_OK;
  } catch (const std::exception&) {
    return DET_E_NOMEM;
  }
}

det_status det_server_poll(det_server* s, int64_t request_id, int timeout_ms, int* done, int* sign,
                           uint32_t* mag, int64_t limb_cap, int64_t* limb_count,
                           double* latency_ms) {
  if (!s || !done) return DET_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(request_id);
  if (it == s->all.end()) return DET_E_INVALID;
  Request* r = it->second.get();
  if (timeout_ms != 0) {
    auto ready = [&] { return r->state == 2; };
    if (timeout_ms < 0) s->cv_done.wait(lk, ready);
    else s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  }
  *done = r->state == 2;
  if (!*done) return DET_OK;
  if (latency_ms) *latency_ms = r->t_done - r->t_submit;
  if (r->status != DET_OK) return r->status;
  if (sign) *sign = r->sign;
  if (limb_count) *limb_count = (int64_t)r->mag.size();
  if ((int64_t)r->mag.size() > limb_cap) return DET_E_BUFFER_TOO_SMALL;
  if (!r->mag.empty() && mag) memcpy(mag, r->mag.data(), r->mag.size() * sizeof(uint32_t));
  return DET_OK;
}

det_status det_server_stats(det_server* s, det_server_report* out) {
  if (!s || !out) return DET_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  out->submitted = s->next_id;
  out->completed = s->completed;
  out->waiting = (int64_t)s->waiting.size();
  out->admitted = (int64_t)s->admitted.size();
  out->max_admitted = s->max_admitted;
  out->rounds = s->rounds;
  out->queue_items = s->queue_items;
  out->hbm_budget = (int64_t)s->budget;
  out->hbm_in_use = (int64_t)s->used;
  out->hbm_peak = (int64_t)s->peak;
  return DET_OK;
}

void det_server_destroy(det_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->engine.joinable()) s->engine.join();
  for (auto& kv : s->all) release(s, kv.second.get());
  delete s;
}

}  // extern "C"
