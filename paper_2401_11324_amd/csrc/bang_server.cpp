// Continuous-batching request loop over one index (see bang.h,
// bang_server_*).  Requests (nq queries with their own k and L) queue on
// the host; a scheduler thread packs the oldest ones into a mixed batch as
// soon as one of the slots is free, and launches it: each slot owns a HIP
// stream, a search workspace and pinned staging buffers, so batches on
// different slots run on the device at the same time and a request that
// arrives while others are searched starts as soon as a slot frees up.
// A batch is one persistent search launch with per-query (k, L): every
// query's result equals a search of that query alone.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "api_internal.h"

using bang::fail;
using bang::hip_fail;
using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  uint64_t ticket = 0;
  uint32_t nq = 0, k = 0, L = 0;
  std::vector<unsigned char> queries;  // nq rows, copied at submit
  std::vector<uint32_t> ids;           // nq x k once done
  std::vector<float> dists;
  Clock::time_point done_at;
  int status = 1;  // 1 pending, 0 done, < 0 failed (BANG_E*)
  std::string error;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bang::Workspace ws;
  void* d_q = nullptr;       // [max_batch][row]
  uint32_t* d_L = nullptr;   // [max_batch]
  uint32_t* d_k = nullptr;
  uint32_t* d_ids = nullptr; // [max_batch][max_k]
  float* d_d = nullptr;
  unsigned char* h_q = nullptr;  // pinned staging of the same
  uint32_t* h_L = nullptr;
  uint32_t* h_k = nullptr;
  uint32_t* h_ids = nullptr;
  float* h_d = nullptr;
  std::vector<std::shared_ptr<Request>> batch;
  uint32_t kb = 0;  // row stride of this batch's results
  bool busy = false;
  // BANG_SERVER_GRAPHS: the batch's copies and search captured once per
  // (bucket of queries, k, L) and replayed; key bucket | k << 21 | L << 42
  std::unordered_map<uint64_t, hipGraphExec_t> graphs;
};

}  // namespace

struct bang_server {
  bang_index* ix = nullptr;
  bang_server_opts o{};
  size_t row = 0;  // bytes per query
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable work_cv;  // new request or stop
  std::condition_variable done_cv;  // a request completed
  std::deque<std::shared_ptr<Request>> pending;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> live;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  // statistics
  uint64_t launches = 0, queries = 0, max_in_flight = 0, requests = 0;
};

namespace {

void free_slot(Slot& s) {
  if (s.stream) (void)hipStreamSynchronize(s.stream);
  for (auto& g : s.graphs) (void)hipGraphExecDestroy(g.second);
  s.graphs.clear();
  bang::workspace_free(&s.ws);
  (void)hipFree(s.d_q);
  (void)hipFree(s.d_L);
  (void)hipFree(s.d_k);
  (void)hipFree(s.d_ids);
  (void)hipFree(s.d_d);
  if (s.h_q) (void)hipHostFree(s.h_q);
  if (s.h_L) (void)hipHostFree(s.h_L);
  if (s.h_k) (void)hipHostFree(s.h_k);
  if (s.h_ids) (void)hipHostFree(s.h_ids);
  if (s.h_d) (void)hipHostFree(s.h_d);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot{};
}

int init_slot(bang_server* sv, Slot& s, size_t ws_bytes) {
  const uint32_t B = sv->o.max_batch, K = sv->o.max_k;
  hipError_t e;
  // default stream priority (the only one used anywhere here)
  if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) ||
      (e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)))
    return hip_fail(e, "server stream");
  int rc = bang::workspace_init(&s.ws, ws_bytes);
  if (rc) return rc;
  if ((e = hipMalloc(&s.d_q, B * sv->row)) ||
      (e = hipMalloc(reinterpret_cast<void**>(&s.d_L), B * 4)) ||
      (e = hipMalloc(reinterpret_cast<void**>(&s.d_k), B * 4)) ||
      (e = hipMalloc(reinterpret_cast<void**>(&s.d_ids), (size_t)B * K * 4)) ||
      (e = hipMalloc(reinterpret_cast<void**>(&s.d_d), (size_t)B * K * 4)))
    return fail(BANG_ENOMEM, std::string("server slot buffers: ") +
                                 hipGetErrorString(e));
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&s.h_q), B * sv->row,
                         hipHostMallocDefault)) ||
      (e = hipHostMalloc(reinterpret_cast<void**>(&s.h_L), B * 4,
                         hipHostMallocDefault)) ||
      (e = hipHostMalloc(reinterpret_cast<void**>(&s.h_k), B * 4,
                         hipHostMallocDefault)) ||
      (e = hipHostMalloc(reinterpret_cast<void**>(&s.h_ids), (size_t)B * K * 4,
                         hipHostMallocDefault)) ||
      (e = hipHostMalloc(reinterpret_cast<void**>(&s.h_d), (size_t)B * K * 4,
                         hipHostMallocDefault)))
    return fail(BANG_ENOMEM, std::string("server pinned buffers: ") +
                                 hipGetErrorString(e));
  // graph buckets search padding rows too: defined (zero) queries
  std::memset(s.h_q, 0, B * sv->row);
  return BANG_OK;
}

void fail_batch(bang_server* sv, Slot& s, int code, const std::string& why) {
  std::lock_guard<std::mutex> g(sv->mu);
  for (auto& r : s.batch) {
    r->status = code;
    r->error = why;
    r->done_at = Clock::now();
  }
  s.batch.clear();
  s.busy = false;
  sv->done_cv.notify_all();
}

// Enqueue a staged batch's copies in, search and copies back, n queries
// with result stride kb and worklists up to Lb, on the slot's stream.
int enqueue(bang_server* sv, Slot& s, uint32_t n, uint32_t kb, uint32_t Lb) {
  hipError_t e;
  if ((e = hipMemcpyAsync(s.d_q, s.h_q, (size_t)n * sv->row,
                          hipMemcpyHostToDevice, s.stream)) ||
      (e = hipMemcpyAsync(s.d_L, s.h_L, (size_t)n * 4, hipMemcpyHostToDevice,
                          s.stream)) ||
      (e = hipMemcpyAsync(s.d_k, s.h_k, (size_t)n * 4, hipMemcpyHostToDevice,
                          s.stream)))
    return hip_fail(e, "server copy in");
  bang_search_opts so{};
  so.table = sv->o.table;
  so.query_L = s.d_L;
  so.query_k = s.d_k;
  int rc = bang::search_with(sv->ix, &s.ws, false, s.d_q, n, kb, Lb, s.d_ids,
                             s.d_d, &so, s.stream);
  if (rc) return rc;
  if ((e = hipMemcpyAsync(s.h_ids, s.d_ids, (size_t)n * kb * 4,
                          hipMemcpyDeviceToHost, s.stream)) ||
      (e = hipMemcpyAsync(s.h_d, s.d_d, (size_t)n * kb * 4,
                          hipMemcpyDeviceToHost, s.stream)))
    return hip_fail(e, "server copy out");
  return BANG_OK;
}

// The batch as one graph launch: n queries rounded up to a bucket (a power
// of two, at most max_batch), the rows past n searched with L = k = 1 (a
// single expansion; their results are not read).  Each (bucket, kb, Lb)
// is captured the first time it occurs and replayed after that; the search
// leaves its counters at zero, so a replay needs no reset.
void launch_graph(bang_server* sv, Slot& s, uint32_t n, uint32_t kb,
                  uint32_t Lb) {
  uint32_t nb = 1;
  while (nb < n) nb <<= 1;
  nb = std::min(nb, sv->o.max_batch);
  for (uint32_t i = n; i < nb; ++i) s.h_L[i] = s.h_k[i] = 1;
  const uint64_t key = (uint64_t)nb | ((uint64_t)kb << 21) |
                       ((uint64_t)Lb << 42);
  hipError_t e;
  auto it = s.graphs.find(key);
  if (it == s.graphs.end()) {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    e = hipStreamBeginCapture(s.stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      fail_batch(sv, s, BANG_EDEVICE, hipGetErrorString(e));
      return;
    }
    const int rc = enqueue(sv, s, nb, kb, Lb);
    const std::string why = rc ? bang::last_error() : std::string();
    e = hipStreamEndCapture(s.stream, &g);
    if (rc || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      fail_batch(sv, s, rc ? rc : BANG_EDEVICE,
                 rc ? why : std::string(hipGetErrorString(e)));
      return;
    }
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      fail_batch(sv, s, BANG_EDEVICE, hipGetErrorString(e));
      return;
    }
    it = s.graphs.emplace(key, x).first;
  }
  if ((e = hipGraphLaunch(it->second, s.stream)) ||
      (e = hipEventRecord(s.done, s.stream))) {
    fail_batch(sv, s, BANG_EDEVICE, hipGetErrorString(e));
    return;
  }
  std::lock_guard<std::mutex> g(sv->mu);
  sv->launches++;
  sv->queries += n;
}

// Stage a batch into the slot and enqueue copies, search and copies back.
void launch(bang_server* sv, Slot& s) {
  uint32_t n = 0, kb = 1, Lb = 1;
  for (auto& r : s.batch) {
    std::memcpy(s.h_q + (size_t)n * sv->row, r->queries.data(),
                (size_t)r->nq * sv->row);
    for (uint32_t i = 0; i < r->nq; ++i) {
      s.h_L[n + i] = r->L;
      s.h_k[n + i] = r->k;
    }
    n += r->nq;
    kb = std::max(kb, r->k);
    Lb = std::max(Lb, r->L);
  }
  s.kb = kb;
  if (sv->o.flags & BANG_SERVER_GRAPHS) {
    launch_graph(sv, s, n, kb, Lb);
    return;
  }
  hipError_t e;
  if ((e = hipMemcpyAsync(s.d_q, s.h_q, (size_t)n * sv->row,
                          hipMemcpyHostToDevice, s.stream)) ||
      (e = hipMemcpyAsync(s.d_L, s.h_L, (size_t)n * 4, hipMemcpyHostToDevice,
                          s.stream)) ||
      (e = hipMemcpyAsync(s.d_k, s.h_k, (size_t)n * 4, hipMemcpyHostToDevice,
                          s.stream))) {
    fail_batch(sv, s, BANG_EDEVICE, hipGetErrorString(e));
    return;
  }
  bang_search_opts so{};
  so.table = sv->o.table;
  so.query_L = s.d_L;
  so.query_k = s.d_k;
  int rc = bang::search_with(sv->ix, &s.ws, false, s.d_q, n, kb, Lb, s.d_ids,
                             s.d_d, &so, s.stream);
  if (rc) {
    fail_batch(sv, s, rc, bang::last_error());
    return;
  }
  if ((e = hipMemcpyAsync(s.h_ids, s.d_ids, (size_t)n * kb * 4,
                          hipMemcpyDeviceToHost, s.stream)) ||
      (e = hipMemcpyAsync(s.h_d, s.d_d, (size_t)n * kb * 4,
                          hipMemcpyDeviceToHost, s.stream)) ||
      (e = hipEventRecord(s.done, s.stream))) {
    fail_batch(sv, s, BANG_EDEVICE, hipGetErrorString(e));
    return;
  }
  std::lock_guard<std::mutex> g(sv->mu);
  sv->launches++;
  sv->queries += n;
}

// Results of a finished slot back to its requests.
void finish(bang_server* sv, Slot& s) {
  const auto now = Clock::now();
  uint32_t off = 0;
  for (auto& r : s.batch) {
    r->ids.resize((size_t)r->nq * r->k);
    r->dists.resize((size_t)r->nq * r->k);
    for (uint32_t i = 0; i < r->nq; ++i) {
      std::memcpy(&r->ids[(size_t)i * r->k], s.h_ids + (size_t)(off + i) * s.kb,
                  r->k * 4);
      std::memcpy(&r->dists[(size_t)i * r->k], s.h_d + (size_t)(off + i) * s.kb,
                  r->k * 4);
    }
    off += r->nq;
  }
  std::lock_guard<std::mutex> g(sv->mu);
  for (auto& r : s.batch) {
    r->done_at = now;
    r->status = 0;
  }
  s.batch.clear();
  s.busy = false;
  sv->done_cv.notify_all();
}

void run(bang_server* sv) {
  (void)hipSetDevice(sv->ix->device);
  for (;;) {
    // completions
    uint64_t in_flight = 0;
    for (auto& s : sv->slots) {
      if (!s.busy) continue;
      hipError_t e = hipEventQuery(s.done);
      if (e == hipSuccess)
        finish(sv, s);
      else if (e != hipErrorNotReady)
        fail_batch(sv, s, BANG_EDEVICE, hipGetErrorString(e));
      else
        ++in_flight;
    }
    // admission: the oldest requests, as many as fit one launch, into
    // every free slot
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->max_in_flight = std::max(sv->max_in_flight, in_flight);
    bool launched = false;
    for (auto& s : sv->slots) {
      if (s.busy || sv->pending.empty()) continue;
      uint32_t n = 0;
      while (!sv->pending.empty() &&
             n + sv->pending.front()->nq <= sv->o.max_batch) {
        n += sv->pending.front()->nq;
        s.batch.push_back(std::move(sv->pending.front()));
        sv->pending.pop_front();
      }
      s.busy = true;
      lk.unlock();
      launch(sv, s);
      launched = true;
      lk.lock();
    }
    bool any_busy = false;
    for (auto& s : sv->slots) any_busy = any_busy || s.busy;
    if (sv->stop && sv->pending.empty() && !any_busy) break;
    if (launched) continue;
    if (!any_busy) {
      sv->work_cv.wait(lk, [&] { return sv->stop || !sv->pending.empty(); });
    } else {
      // work on the device: poll its events, wake early for new requests
      sv->work_cv.wait_for(lk, std::chrono::microseconds(20), [&] {
        if (sv->pending.empty()) return false;
        for (auto& s : sv->slots)
          if (!s.busy) return true;
        return false;
      });
    }
  }
}

int submit(bang_server* sv, const void* queries, uint32_t nq, uint32_t k,
           uint32_t L, uint64_t* ticket) {
  if (!sv || !ticket) return fail(BANG_EINVAL, "null argument");
  if (nq == 0 || nq > sv->o.max_batch)
    return fail(BANG_EINVAL, "need 1 <= nq <= max_batch");
  if (!queries) return fail(BANG_EINVAL, "null queries");
  if (k < 1 || k > L || k > sv->o.max_k || L > sv->o.max_L)
    return fail(BANG_EINVAL, "need 1 <= k <= L, k <= max_k, L <= max_L");
  if (k > sv->ix->dev.n) return fail(BANG_EINVAL, "k > n");
  auto r = std::make_shared<Request>();
  r->nq = nq;
  r->k = k;
  r->L = L;
  r->queries.assign(static_cast<const unsigned char*>(queries),
                    static_cast<const unsigned char*>(queries) +
                        (size_t)nq * sv->row);
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (sv->stop) return fail(BANG_EABORTED, "server is shutting down");
    r->ticket = sv->next_ticket++;
    sv->live[r->ticket] = r;
    sv->pending.push_back(r);
    sv->requests++;
  }
  sv->work_cv.notify_one();
  *ticket = r->ticket;
  return BANG_OK;
}

int wait_for(bang_server* sv, uint64_t ticket, uint32_t* ids, float* dists,
             int timeout_ms, Clock::time_point* done_at) {
  if (!sv) return fail(BANG_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  std::shared_ptr<Request> r;
  {
    auto it = sv->live.find(ticket);
    if (it == sv->live.end()) return fail(BANG_EINVAL, "unknown ticket");
    r = it->second;  // no iterator is kept: the wait releases the lock
  }
  auto ready = [&] { return r->status <= 0; };
  if (timeout_ms < 0) {
    sv->done_cv.wait(lk, ready);
  } else if (!sv->done_cv.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                                   ready)) {
    return fail(BANG_EABORTED, "timed out; the request is still queued");
  }
  // another thread waiting on the same ticket may have collected it
  if (sv->live.erase(ticket) == 0)
    return fail(BANG_EINVAL, "ticket already collected by another wait");
  lk.unlock();
  if (r->status < 0) return fail(r->status, r->error);
  if (ids) std::memcpy(ids, r->ids.data(), r->ids.size() * 4);
  if (dists) std::memcpy(dists, r->dists.data(), r->dists.size() * 4);
  if (done_at) *done_at = r->done_at;
  return BANG_OK;
}

void shutdown(bang_server* sv) {
  {
    std::lock_guard<std::mutex> g(sv->mu);
    sv->stop = true;
  }
  sv->work_cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  for (auto& s : sv->slots) free_slot(s);
}

}  // namespace

extern "C" {

int bang_server_create(bang_index* ix, const bang_server_opts* o,
                       bang_server** out) {
  try {
    if (!ix || !o || !out) return fail(BANG_EINVAL, "null argument");
    *out = nullptr;
    if (o->max_batch < 1 || o->max_batch > (1u << 20))
      return fail(BANG_EINVAL, "need 1 <= max_batch <= 2^20");
    if (o->slots < 1 || o->slots > 8)
      return fail(BANG_EINVAL, "need 1 <= slots <= 8");
    if (o->max_L < 1 || o->max_L > BANG_MAX_L || o->max_k < 1 ||
        o->max_k > o->max_L)
      return fail(BANG_EINVAL, "need 1 <= max_k <= max_L <= 1024");
    if (o->table > BANG_TABLE_EXACT) return fail(BANG_EINVAL, "unknown table form");
    if (o->flags & ~BANG_SERVER_GRAPHS)
      return fail(BANG_EINVAL, "unknown server flags");
    hipError_t e = hipSetDevice(ix->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const uint32_t cap = std::max(4 * o->max_L, o->max_L + 64);
    const size_t ws = bang::search_workspace_bytes(ix, o->max_batch, o->max_L,
                                                   cap, o->table);
    if (ws == 0) return BANG_EUNSUPPORTED;  // message set
    auto sv = std::make_unique<bang_server>();
    sv->ix = ix;
    sv->o = *o;
    sv->row = (size_t)ix->dev.d * (ix->dev.dtype == BANG_F32 ? 4 : 1);
    // admission by memory: as many slots as the budget holds
    const size_t per_slot = ws + (size_t)o->max_batch *
                                     (sv->row + 8 + 8 * (size_t)o->max_k);
    uint32_t nslots = o->slots;
    if (o->hbm_budget_bytes) {
      const uint64_t fit = o->hbm_budget_bytes / per_slot;
      if (fit == 0)
        return fail(BANG_ENOMEM, "one slot needs " + std::to_string(per_slot) +
                                     " bytes, over the budget");
      nslots = (uint32_t)std::min<uint64_t>(nslots, fit);
    }
    sv->slots.resize(nslots);
    for (auto& s : sv->slots) {
      int rc = init_slot(sv.get(), s, ws);
      if (rc) {
        for (auto& t : sv->slots) free_slot(t);
        return rc;
      }
    }
    sv->worker = std::thread(run, sv.get());
    *out = sv.release();
    return BANG_OK;
  } catch (const std::exception& ex) {
    return fail(BANG_ENOMEM, ex.what());
  }
}

int bang_server_destroy(bang_server* sv) {
  if (!sv) return BANG_OK;
  try {
    shutdown(sv);
  } catch (...) {
  }
  delete sv;
  return BANG_OK;
}

int bang_server_submit(bang_server* sv, const void* queries, uint32_t nq,
                       uint32_t k, uint32_t L, uint64_t* ticket) {
  try {
    return submit(sv, queries, nq, k, L, ticket);
  } catch (const std::exception& ex) {
    return fail(BANG_ENOMEM, ex.what());
  }
}

int bang_server_wait(bang_server* sv, uint64_t ticket, uint32_t* ids,
                     float* dists, int timeout_ms) {
  try {
    return wait_for(sv, ticket, ids, dists, timeout_ms, nullptr);
  } catch (const std::exception& ex) {
    return fail(BANG_ENOMEM, ex.what());
  }
}

int bang_server_replay(bang_server* sv, const void* queries, uint32_t nreq,
                       const uint32_t* nq, const uint32_t* k,
                       const uint32_t* L, const double* arrival_s,
                       uint32_t kstride, uint32_t* ids, float* dists,
                       double* latency_s) {
  try {
    if (!sv || !queries || !nq || !k || !L || !arrival_s || !ids || !dists ||
        !latency_s)
      return fail(BANG_EINVAL, "null argument");
    for (uint32_t j = 0; j < nreq; ++j) {
      if (k[j] > kstride) return fail(BANG_EINVAL, "k above kstride");
      if (j && arrival_s[j] < arrival_s[j - 1])
        return fail(BANG_EINVAL, "arrival times must not decrease");
    }
    std::vector<uint64_t> tickets(nreq, 0);
    const auto t0 = Clock::now();
    size_t off = 0;
    for (uint32_t j = 0; j < nreq; ++j) {
      std::this_thread::sleep_until(
          t0 + std::chrono::duration_cast<Clock::duration>(
                   std::chrono::duration<double>(arrival_s[j])));
      int rc = submit(sv, static_cast<const unsigned char*>(queries) +
                              off * sv->row,
                      nq[j], k[j], L[j], &tickets[j]);
      if (rc) return rc;
      off += nq[j];
    }
    std::vector<uint32_t> bi;
    std::vector<float> bd;
    off = 0;
    int first_err = BANG_OK;
    for (uint32_t j = 0; j < nreq; ++j) {
      bi.resize((size_t)nq[j] * k[j]);
      bd.resize((size_t)nq[j] * k[j]);
      Clock::time_point done;
      int rc = wait_for(sv, tickets[j], bi.data(), bd.data(), -1, &done);
      if (rc && !first_err) first_err = rc;
      for (uint32_t i = 0; i < nq[j]; ++i)
        for (uint32_t c = 0; c < kstride; ++c) {
          const bool in = !rc && c < k[j];
          ids[(off + i) * kstride + c] = in ? bi[(size_t)i * k[j] + c] : BANG_NONE;
          dists[(off + i) * kstride + c] =
              in ? bd[(size_t)i * k[j] + c] : __builtin_inff();
        }
      latency_s[j] =
          rc ? -1.0
             : std::chrono::duration<double>(done - t0).count() - arrival_s[j];
      off += nq[j];
    }
    return first_err;
  } catch (const std::exception& ex) {
    return fail(BANG_ENOMEM, ex.what());
  }
}

int bang_server_stats(bang_server* sv, uint64_t* out, uint32_t n) {
  if (!sv || !out) return fail(BANG_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(sv->mu);
  const uint64_t v[5] = {sv->requests, sv->launches, sv->queries,
                         sv->max_in_flight, (uint64_t)sv->slots.size()};
  for (uint32_t i = 0; i < n && i < 5; ++i) out[i] = v[i];
  return BANG_OK;
}

}  // extern "C"
