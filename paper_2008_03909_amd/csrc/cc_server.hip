// Serving loop for batch-incremental connectivity: continuous batching of
// Insert and IsConnected requests over one device-resident union-find state.
//
// Semantics (the batch-incremental correctness of ConnectIt's streaming
// appendix, with arrival order as the batch order): a query request sees
// exactly the insert requests that arrived before it.  Inserts commute with
// inserts and queries with queries, so consecutive requests of one type form
// a phase whose requests run concurrently on several HIP streams; at a change
// of type a barrier event (recorded after every request of the previous
// phase) orders the new phase after the old one.  Requests are admitted in
// arrival order when their device bytes fit in the memory budget and a
// stream slot is free, so new work starts while older work is still running.
//
// Host side: zero copy -- request payloads are DMA'd straight from the
// caller's buffers (which must stay valid until the request completes; pinned
// memory makes the copies asynchronous) and query answers land directly in
// the caller's output buffer.  Device side: a first-fit pool of the budget.
// Latency = completion (observed by polling the request's event) minus
// arrival, on the host's steady clock.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <vector>

#include "cc_device.h"
#include "cc_internal.h"
#include "cc_static.h"

struct cc_stream;  // defined in cc_stream.hip; used only through the C ABI

namespace cc {

// First-fit allocator over [0, size) with coalescing frees.
class RangePool {
 public:
  explicit RangePool(size_t size = 0) { reset(size); }
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes ? bytes : 1);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t used() const { return used_; }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0, used_ = 0;
};

struct Request {
  int64_t id = 0;
  int type = 0;  // 0 insert, 1 query
  int64_t k = 0;
  double arrival = 0.0;   // seconds on the server clock
  double admitted = 0.0;
  double done_at = -1.0;
  size_t bytes = 0, off = 0;
  int stream = -1;
  hipEvent_t ev = nullptr;
  uint8_t* out_host = nullptr;  // caller's result buffer (queries)
  const int32_t* a = nullptr;   // caller's payload (valid until completion)
  const int32_t* b = nullptr;
  int state = 0;                // 0 pending, 1 in flight, 2 done
};

}  // namespace cc

struct cc_server {
  cc_ctx* ctx = nullptr;
  cc_stream* st = nullptr;
  int64_t n = 0;
  size_t budget = 0;
  int nstreams = 0;
  int max_inflight = 0;
  char* dpool = nullptr;
  cc::RangePool pool;
  std::vector<hipStream_t> streams;
  std::vector<int> stream_busy;  // requests in flight per stream
  hipStream_t barrier_stream = nullptr;
  std::vector<hipEvent_t> events;      // every event created; destroyed with the server
  std::deque<cc::Request*> pending;   // arrival order, not yet admitted
  std::vector<cc::Request*> inflight;
  std::vector<cc::Request*> all;
  // phase bookkeeping
  int phase_type = -1;
  hipEvent_t phase_barrier = nullptr;       // previous phases complete
  std::vector<hipEvent_t> phase_events;     // completion events of the current phase
  std::chrono::steady_clock::time_point t0;
  int64_t next_id = 0;
  uint32_t device_error = 0;
};

namespace cc {

static double now_s(const cc_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

static hipEvent_t take_event(cc_server* s) {
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  s->events.push_back(e);
  return e;
}

// Closes the current phase: a barrier event on the barrier stream after every
// completion event of the phase.
static cc_status close_phase(cc_server* s) {
  for (hipEvent_t e : s->phase_events) CC_HIP(hipStreamWaitEvent(s->barrier_stream, e, 0));
  hipEvent_t b = take_event(s);
  if (!b) return fail(CC_EDEVICE, "cannot create an event");
  CC_HIP(hipEventRecord(b, s->barrier_stream));
  s->phase_barrier = b;
  s->phase_events.clear();
  return CC_OK;
}

static cc_status launch(cc_server* s, Request* r) {
  // pick the least loaded stream
  int best = 0;
  for (int i = 1; i < s->nstreams; ++i)
    if (s->stream_busy[i] < s->stream_busy[best]) best = i;
  hipStream_t hs = s->streams[best];
  r->stream = best;
  s->stream_busy[best]++;
  char* d = s->dpool + r->off;
  const size_t half = (size_t)r->k * 4;
  const size_t pair_bytes = 2 * half;
  if (r->type != s->phase_type) {
    if (s->phase_type != -1) {
      cc_status st = close_phase(s);
      if (st != CC_OK) return st;
    }
    s->phase_type = r->type;
  }
  CC_HIP(hipMemcpyAsync(d, r->a, half, hipMemcpyHostToDevice, hs));
  CC_HIP(hipMemcpyAsync(d + half, r->b, half, hipMemcpyHostToDevice, hs));
  if (s->phase_barrier) CC_HIP(hipStreamWaitEvent(hs, s->phase_barrier, 0));
  const int32_t* a = (const int32_t*)d;
  const int32_t* b = (const int32_t*)(d + (size_t)r->k * 4);
  cc_status st;
  if (r->type == 0) {
    st = cc_insert_batch(s->st, r->k, a, b, hs);
  } else {
    uint8_t* out = (uint8_t*)(d + pair_bytes);
    st = cc_query_batch(s->st, r->k, a, b, out, hs);
    if (st == CC_OK) CC_HIP(hipMemcpyAsync(r->out_host, out, (size_t)r->k, hipMemcpyDeviceToHost, hs));
  }
  if (st != CC_OK) return st;
  r->ev = take_event(s);
  if (!r->ev) return fail(CC_EDEVICE, "cannot create an event");
  CC_HIP(hipEventRecord(r->ev, hs));
  s->phase_events.push_back(r->ev);
  r->state = 1;
  r->admitted = now_s(s);
  s->inflight.push_back(r);
  return CC_OK;
}

}  // namespace cc

using namespace cc;

extern "C" {

cc_status cc_server_create(cc_ctx* ctx, int64_t n, const cc_variant* v, int64_t budget_bytes, int num_streams,
                           int max_inflight, cc_server** out) {
  if (!ctx || !out) return fail(CC_EINVAL, "NULL argument");
  *out = nullptr;
  if (budget_bytes < 4096) return fail(CC_EINVAL, "budget below 4 KiB");
  if (num_streams < 1 || num_streams > 16) return fail(CC_EINVAL, "num_streams must be in [1, 16]");
  if (max_inflight < 1 || max_inflight > 1024) return fail(CC_EINVAL, "max_inflight must be in [1, 1024]");
  cc_server* s = new cc_server();
  s->ctx = ctx;
  s->n = n;
  cc_status st = cc_stream_create(ctx, n, v, &s->st);
  if (st != CC_OK) {
    delete s;
    return st;
  }
  s->budget = (size_t)budget_bytes;
  s->nstreams = num_streams;
  s->max_inflight = max_inflight;
  if (hipMalloc((void**)&s->dpool, s->budget) != hipSuccess) {
    cc_stream_destroy(s->st);
    delete s;
    return fail(CC_ENOMEM, "cannot allocate a %lld-byte request pool", (long long)budget_bytes);
  }
  s->pool.reset(s->budget);
  s->streams.resize(num_streams);
  s->stream_busy.assign(num_streams, 0);
  for (auto& x : s->streams) CC_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
  CC_HIP(hipStreamCreateWithFlags(&s->barrier_stream, hipStreamNonBlocking));
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return CC_OK;
}

void cc_server_destroy(cc_server* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  for (auto* r : s->all) delete r;
  for (auto e : s->events) (void)hipEventDestroy(e);
  for (auto x : s->streams) (void)hipStreamDestroy(x);
  if (s->barrier_stream) (void)hipStreamDestroy(s->barrier_stream);
  if (s->dpool) (void)hipFree(s->dpool);
  cc_stream_destroy(s->st);
  delete s;
}

double cc_server_clock(cc_server* s) { return s ? now_s(s) : 0.0; }

static cc_status submit(cc_server* s, int type, int64_t k, const int32_t* a, const int32_t* b, uint8_t* out,
                        double arrival, int64_t* id) {
  if (!s) return fail(CC_EINVAL, "server is NULL");
  if (k < 1) return fail(CC_EINVAL, "a request needs at least one pair");
  if (!a || !b || (type == 1 && !out)) return fail(CC_EINVAL, "NULL array");
  const size_t bytes = (size_t)k * 8 + (type == 1 ? (size_t)k : 0);
  if (align256(bytes) > s->budget)
    return fail(CC_EBUSY, "request of %zu bytes can never fit the %zu-byte budget", bytes, s->budget);
  Request* r = new Request();
  r->id = s->next_id++;
  r->type = type;
  r->k = k;
  r->arrival = arrival >= 0 ? arrival : now_s(s);
  r->bytes = bytes;
  r->out_host = out;
  s->all.push_back(r);
  r->a = a;
  r->b = b;
  s->pending.push_back(r);
  if (id) *id = r->id;
  return CC_OK;
}

cc_status cc_server_submit_insert(cc_server* s, int64_t k, const int32_t* u, const int32_t* v, double arrival,
                                  int64_t* id) {
  return submit(s, 0, k, u, v, nullptr, arrival, id);
}

cc_status cc_server_submit_query(cc_server* s, int64_t q, const int32_t* a, const int32_t* b, uint8_t* out,
                                 double arrival, int64_t* id) {
  return submit(s, 1, q, a, b, out, arrival, id);
}

}  // extern "C"

namespace cc {
// Retires finished requests, then admits pending ones in arrival order while
// memory and stream slots allow.
static cc_status progress_staged(cc_server* s) {
  for (size_t i = 0; i < s->inflight.size();) {
    Request* r = s->inflight[i];
    hipError_t q = hipEventQuery(r->ev);
    if (q == hipSuccess) {
      r->done_at = now_s(s);
      r->state = 2;
      s->pool.release(r->off, r->bytes);
      s->stream_busy[r->stream]--;
      s->inflight[i] = s->inflight.back();
      s->inflight.pop_back();
    } else if (q == hipErrorNotReady) {
      ++i;
    } else {
      return fail(CC_EDEVICE, "request event failed: %s", hipGetErrorString(q));
    }
  }
  while (!s->pending.empty() && (int)s->inflight.size() < s->max_inflight) {
    Request* r = s->pending.front();
    size_t off = 0;
    if (!s->pool.alloc(r->bytes, &off)) break;
    r->off = off;
    s->pending.pop_front();
    cc_status st = launch(s, r);
    if (st != CC_OK) return st;
  }
  return CC_OK;
}
}  // namespace cc

extern "C" {

cc_status cc_server_poll(cc_server* s, int wait_all) {
  if (!s) return fail(CC_EINVAL, "server is NULL");
  do {
    cc_status st = progress_staged(s);
    if (st != CC_OK) return st;
  } while (wait_all && (!s->pending.empty() || !s->inflight.empty()));
  if (wait_all) {
    cc_status st = cc_stream_sync_status(s->st);
    if (st != CC_OK) return st;
  }
  return CC_OK;
}

// Replays a request trace in real time: request i (type[i] 0 = insert,
// 1 = query) arrives at arrival_s[i] seconds after the call starts, carrying
// pairs [start[i], start[i] + len[i]) of the a/b arrays; query answers go to
// out[start[i] ...].  Between arrivals the loop keeps retiring and admitting.
// latency_s[i] receives completion minus arrival.
cc_status cc_server_run_trace(cc_server* s, int64_t count, const int32_t* type, const double* arrival_s,
                              const int64_t* start, const int64_t* len, const int32_t* a, const int32_t* b,
                              uint8_t* out, double* latency_s) {
  if (!s || count < 0 || (count && (!type || !arrival_s || !start || !len || !a || !b || !latency_s)))
    return fail(CC_EINVAL, "bad trace arguments");
  const double base = now_s(s);
  std::vector<int64_t> ids(count);
  for (int64_t i = 0; i < count; ++i) {
    while (now_s(s) - base < arrival_s[i]) {
      cc_status st = progress_staged(s);
      if (st != CC_OK) return st;
    }
    cc_status st = submit(s, type[i] ? 1 : 0, len[i], a + start[i], b + start[i], type[i] ? out + start[i] : nullptr,
                          base + arrival_s[i], &ids[i]);
    if (st != CC_OK) return st;
    st = progress_staged(s);
    if (st != CC_OK) return st;
  }
  cc_status st = cc_server_poll(s, 1);
  if (st != CC_OK) return st;
  for (int64_t i = 0; i < count; ++i) {
    const Request* r = s->all[(size_t)ids[i]];
    latency_s[i] = r->done_at - r->arrival;
  }
  return CC_OK;
}

cc_status cc_server_request_info(cc_server* s, int64_t id, int* done, double* latency_s) {
  if (!s || id < 0 || id >= (int64_t)s->all.size()) return fail(CC_EINVAL, "unknown request");
  const Request* r = s->all[(size_t)id];
  if (done) *done = r->state == 2;
  if (latency_s) *latency_s = r->state == 2 ? r->done_at - r->arrival : -1.0;
  return CC_OK;
}

cc_status cc_server_labels(cc_server* s, int32_t* labels_out, int64_t* num_components_dev, void* hip_stream) {
  if (!s) return fail(CC_EINVAL, "server is NULL");
  cc_status st = cc_server_poll(s, 1);
  if (st != CC_OK) return st;
  return cc_stream_labels(s->st, labels_out, num_components_dev, hip_stream);
}

int64_t cc_server_pool_used(cc_server* s) { return s ? (int64_t)s->pool.used() : -1; }

}  // extern "C"
