// serve.cpp -- a request loop over the codec with continuous batching.
//
// Clients submit compress and decompress requests on device-resident
// inputs from any thread.  A worker thread admits requests in arrival
// order as output memory frees up in a fixed HBM pool (the budget), groups
// the admitted requests of one kind into a batch launch (batch.cpp) on a
// free lane -- a stream with its own batch scratch -- and, while those
// batches run, keeps admitting and launching new arrivals on the other
// lanes, so work from different batches overlaps on the device.  A batch
// completes when its lane's event fires; its requests' outputs stay in the
// pool until the client releases them.
//
// Every request's output is the byte-identical result of the one-series
// call, whatever batch it joined: the batch launch keeps series independent.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "context.hpp"

using namespace falcon_host;

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over one device allocation, 256-byte granules.
class Pool {
 public:
  bool init(size_t bytes, void* external) {
    if (external) {
      base_ = external;
    } else {
      if (hipMalloc(&base_, bytes) != hipSuccess) return false;
      owned_ = true;
    }
    size_ = bytes;
    free_[0] = bytes;
    return true;
  }
  void destroy() {
    if (base_ && owned_) (void)hipFree(base_);
    base_ = nullptr;
  }
  size_t capacity() const { return size_; }
  void* alloc(size_t bytes) {
    const size_t need = (bytes + 255) & ~(size_t)255;
    std::lock_guard<std::mutex> g(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[off + need] = len - need;
      used_[off] = need;
      return static_cast<uint8_t*>(base_) + off;
    }
    return nullptr;
  }
  bool release(void* p) {
    std::lock_guard<std::mutex> g(mu_);
    const size_t off = static_cast<size_t>(static_cast<uint8_t*>(p) - static_cast<uint8_t*>(base_));
    auto u = used_.find(off);
    if (!p || u == used_.end()) return false;
    size_t start = off, len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {  // merge with the following hole
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {  // merge with the preceding hole
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    return true;
  }

 private:
  void* base_ = nullptr;
  bool owned_ = false;
  size_t size_ = 0;
  std::map<size_t, size_t> free_, used_;
  std::mutex mu_;
};

struct Req {
  falcon_request r;
  size_t out_bytes = 0;
  void* out = nullptr;
  double t_submit = 0, t_admit = 0;
};

struct ServeLane {
  hipStream_t stream = nullptr;
  hipEvent_t ev_start = nullptr;  // before the batch's launches
  hipEvent_t ev = nullptr;        // after them
  BatchScratch scratch;
  BatchLayout layout;
  std::vector<Req> reqs;       // the batch in flight
  std::vector<falcon_series> series;
  bool busy = false;
};

}  // namespace

struct falcon_server {
  falcon_ctx* ctx = nullptr;
  falcon_server_opts opts{};
  Pool pool;
  std::vector<ServeLane> lanes;
  Clock::time_point t0;
  std::thread worker;
  std::atomic<bool> stop{false};
  // submission queue (clients -> worker)
  std::mutex in_mu;
  std::condition_variable in_cv;
  std::vector<Req> incoming;
  // completion queue (worker -> clients)
  std::mutex out_mu;
  std::condition_variable out_cv;
  std::deque<falcon_completion> done;
  // worker-only state
  std::deque<Req> pending, admitted;
  std::atomic<uint64_t> in_flight{0};
  hipEvent_t ev_ref = nullptr;  // device time origin of the batch intervals

  double now_us() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }
};

namespace {

size_t output_bytes(const falcon_request& r) {
  if (r.op == FALCON_OP_COMPRESS) return falcon_compress_bound(r.n, r.dtype);
  return r.n * elem_size(r.dtype);
}

// A batch holds at most this many chunks, so that a lane's batch scratch
// (about 36 bytes per chunk, outside the pool) stays below about 150 MB.
constexpr uint64_t kLaneChunkCap = 1ull << 22;

void complete(falcon_server* S, const Req& q, falcon_status st, size_t out_len, int lane = -1,
              double dev_start = -1.0, double dev_end = -1.0) {
  falcon_completion c{};
  c.lane = lane;
  c.dev_start_us = dev_start;
  c.dev_end_us = dev_end;
  c.tag = q.r.tag;
  c.status = st;
  c.d_out = st == FALCON_OK ? q.out : nullptr;
  c.out_len = st == FALCON_OK ? out_len : 0;
  c.submit_us = q.t_submit;
  c.admit_us = q.t_admit;
  c.complete_us = S->now_us();
  if (st != FALCON_OK && q.out) S->pool.release(q.out);
  {
    std::lock_guard<std::mutex> g(S->out_mu);
    S->done.push_back(c);
  }
  S->out_cv.notify_all();
  S->in_flight.fetch_sub(1);
}

falcon_series to_series(const Req& q) {
  falcon_series s{};
  s.d_in = q.r.d_in;
  s.n = q.r.n;
  s.in_len = q.r.in_len;
  s.d_out = q.out;
  s.out_cap = q.out_bytes ? q.out_bytes : 256;
  s.dtype = q.r.dtype;
  return s;
}

// Launches one batch of admitted requests of the same kind on lane L.
void launch_batch(falcon_server* S, ServeLane& L) {
  const int op = S->admitted.front().r.op;
  L.reqs.clear();
  L.series.clear();
  uint64_t chunks = 0;
  for (auto it = S->admitted.begin(); it != S->admitted.end() && (int)L.reqs.size() < S->opts.max_batch;) {
    if (it->r.op != op) {
      ++it;
      continue;
    }
    const uint64_t nc = chunks_of(it->r.n);
    if (!L.reqs.empty() && chunks + nc > kLaneChunkCap) break;
    chunks += nc;
    const falcon_series s = to_series(*it);
    const falcon_status st = batch_check(op, s);
    if (st != FALCON_OK) {
      complete(S, *it, st, 0);
    } else {
      L.reqs.push_back(*it);
      L.series.push_back(s);
    }
    it = S->admitted.erase(it);
  }
  if (L.reqs.empty()) return;
  falcon_status st = batch_layout(L.scratch, op, L.series.data(), L.series.size(), L.layout, L.stream);
  if (st == FALCON_OK) st = dev_err(hipEventRecord(L.ev_start, L.stream));
  if (st == FALCON_OK) st = batch_enqueue(S->ctx, L.scratch, L.layout, BatchGeom(), L.stream, true);
  if (st == FALCON_OK) st = dev_err(hipEventRecord(L.ev, L.stream));
  if (st != FALCON_OK) {
    (void)hipStreamSynchronize(L.stream);
    for (const Req& q : L.reqs) complete(S, q, st, 0);
    L.reqs.clear();
    return;
  }
  L.busy = true;
}

// A batch that reported a corrupt stream is re-run one request at a time,
// so that only the corrupt requests fail.
void finish_batch(falcon_server* S, ServeLane& L) {
  L.busy = false;
  falcon_status st = batch_result(L.scratch, L.layout, L.series.data(), L.series.data());
  if (st == FALCON_OK) {
    // the batch's device interval, from the server's time origin
    float a = -1.f, b = -1.f;
    const int lane = (int)(&L - S->lanes.data());
    if (hipEventElapsedTime(&a, S->ev_ref, L.ev_start) != hipSuccess ||
        hipEventElapsedTime(&b, S->ev_ref, L.ev) != hipSuccess)
      a = b = -1.f;
    for (size_t i = 0; i < L.reqs.size(); ++i)
      complete(S, L.reqs[i], FALCON_OK, L.series[i].out_len, lane, a * 1e3, b * 1e3);
  } else if (st == FALCON_ERR_CORRUPT_STREAM && L.reqs.size() > 1) {
    for (size_t i = 0; i < L.reqs.size(); ++i) {
      BatchLayout one;
      falcon_series s = L.series[i];
      falcon_status r = batch_layout(L.scratch, L.layout.op, &s, 1, one, L.stream);
      if (r == FALCON_OK) r = batch_enqueue(S->ctx, L.scratch, one, BatchGeom(), L.stream, true);
      if (r == FALCON_OK) r = dev_err(hipStreamSynchronize(L.stream));
      if (r == FALCON_OK) r = batch_result(L.scratch, one, &s, &s);
      complete(S, L.reqs[i], r, s.out_len);
    }
  } else {
    for (const Req& q : L.reqs) complete(S, q, st, 0);
  }
  L.reqs.clear();
  L.series.clear();
}

void worker_main(falcon_server* S) {
  (void)hipSetDevice(S->ctx->device);
  for (;;) {
    // 1. completions
    bool busy = false;
    for (auto& L : S->lanes) {
      if (!L.busy) continue;
      const hipError_t e = hipEventQuery(L.ev);
      if (e == hipSuccess) {
        finish_batch(S, L);
      } else if (e != hipErrorNotReady) {
        (void)hipStreamSynchronize(L.stream);
        L.busy = false;
        for (const Req& q : L.reqs) complete(S, q, FALCON_ERR_DEVICE, 0);
        L.reqs.clear();
      }
      busy |= L.busy;
    }
    // 2. new arrivals; sleep when there is nothing to do until a submit, a
    // release or destruction wakes the loop
    bool stopping = false;
    {
      std::unique_lock<std::mutex> g(S->in_mu);
      if (!busy && S->admitted.empty() && S->incoming.empty()) {
        if (S->stop.load()) stopping = true;
        else S->in_cv.wait_for(g, std::chrono::milliseconds(2));
      }
      for (auto& q : S->incoming) S->pending.push_back(q);
      S->incoming.clear();
    }
    // 3. admission in arrival order, as pool memory allows
    while (!S->pending.empty()) {
      Req& q = S->pending.front();
      if (q.out_bytes > S->pool.capacity()) {
        complete(S, q, FALCON_ERR_OUT_OF_MEMORY, 0);
        S->pending.pop_front();
        continue;
      }
      q.out = S->pool.alloc(q.out_bytes ? q.out_bytes : 256);
      if (!q.out) break;  // wait for releases
      q.t_admit = S->now_us();
      S->admitted.push_back(q);
      S->pending.pop_front();
    }
    // 4. launches on free lanes
    for (auto& L : S->lanes) {
      if (S->admitted.empty()) break;
      if (!L.busy) launch_batch(S, L);
    }
    bool any = false;
    for (auto& L : S->lanes) any |= L.busy;
    if (stopping && !any && S->admitted.empty()) {
      // what is still pending cannot be admitted: the pool is held by
      // outputs nobody will release any more
      for (const Req& q : S->pending) complete(S, q, FALCON_ERR_OUT_OF_MEMORY, 0);
      S->pending.clear();
      break;
    }
    if (any && S->admitted.empty()) std::this_thread::sleep_for(std::chrono::microseconds(5));
  }
}

}  // namespace

extern "C" {

falcon_status falcon_server_create(falcon_ctx* ctx, const falcon_server_opts* opts, falcon_server** out) {
  if (!ctx || !out) return FALCON_ERR_INVALID_ARG;
  *out = nullptr;
  falcon_server_opts o{};
  o.hbm_budget = (size_t)64 << 30;
  o.lanes = 4;
  o.max_batch = 256;
  if (opts) {
    o.pool = opts->pool;
    if (opts->hbm_budget) o.hbm_budget = opts->hbm_budget;
    if (opts->lanes) o.lanes = opts->lanes;
    if (opts->max_batch) o.max_batch = opts->max_batch;
  }
  if (o.lanes < 1 || o.lanes > 32 || o.max_batch < 1 || o.hbm_budget < 4096 || ((uintptr_t)o.pool % 256))
    return FALCON_ERR_INVALID_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return FALCON_ERR_DEVICE;
  falcon_server* S = new (std::nothrow) falcon_server();
  if (!S) return FALCON_ERR_OUT_OF_MEMORY;
  S->ctx = ctx;
  S->opts = o;
  S->t0 = Clock::now();
  if (!S->pool.init(o.hbm_budget, o.pool)) {
    delete S;
    return FALCON_ERR_OUT_OF_MEMORY;
  }
  S->lanes.resize((size_t)o.lanes);
  for (auto& L : S->lanes) {
    if (hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreate(&L.ev_start) != hipSuccess || hipEventCreate(&L.ev) != hipSuccess) {
      falcon_server_destroy(S);
      return FALCON_ERR_DEVICE;
    }
  }
  if (hipEventCreate(&S->ev_ref) != hipSuccess || hipEventRecord(S->ev_ref, S->lanes[0].stream) != hipSuccess ||
      hipEventSynchronize(S->ev_ref) != hipSuccess) {
    falcon_server_destroy(S);
    return FALCON_ERR_DEVICE;
  }
  S->worker = std::thread(worker_main, S);
  *out = S;
  return FALCON_OK;
}

falcon_status falcon_server_submit(falcon_server* S, const falcon_request* r) {
  if (!S || !r || (r->op != FALCON_OP_COMPRESS && r->op != FALCON_OP_DECOMPRESS) || elem_size(r->dtype) == 0)
    return FALCON_ERR_INVALID_ARG;
  Req q;
  q.r = *r;
  q.out_bytes = output_bytes(*r);
  q.t_submit = S->now_us();
  S->in_flight.fetch_add(1);
  {
    std::lock_guard<std::mutex> g(S->in_mu);
    S->incoming.push_back(q);
  }
  S->in_cv.notify_one();
  return FALCON_OK;
}

size_t falcon_server_poll(falcon_server* S, falcon_completion* out, size_t max, int wait_ms) {
  if (!S || !out || max == 0) return 0;
  std::unique_lock<std::mutex> g(S->out_mu);
  if (S->done.empty() && wait_ms > 0)
    S->out_cv.wait_for(g, std::chrono::milliseconds(wait_ms), [S] { return !S->done.empty(); });
  size_t k = 0;
  while (k < max && !S->done.empty()) {
    out[k++] = S->done.front();
    S->done.pop_front();
  }
  return k;
}

falcon_status falcon_server_release(falcon_server* S, void* d_out) {
  if (!S || !d_out) return FALCON_ERR_INVALID_ARG;
  if (!S->pool.release(d_out)) return FALCON_ERR_INVALID_ARG;
  S->in_cv.notify_one();  // admission may proceed
  return FALCON_OK;
}

uint64_t falcon_server_in_flight(const falcon_server* S) { return S ? S->in_flight.load() : 0; }

void falcon_server_destroy(falcon_server* S) {
  if (!S) return;
  if (S->worker.joinable()) {  // the worker finishes what it can and exits
    S->stop.store(true);
    S->in_cv.notify_all();
    S->worker.join();
  }
  (void)hipSetDevice(S->ctx->device);
  for (auto& L : S->lanes) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    batch_free(L.scratch);
    if (L.ev_start) (void)hipEventDestroy(L.ev_start);
    if (L.ev) (void)hipEventDestroy(L.ev);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
  if (S->ev_ref) (void)hipEventDestroy(S->ev_ref);
  S->pool.destroy();
  delete S;
}

}  // extern "C"
