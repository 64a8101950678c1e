// Serving loop for batch-incremental connectivity: continuous batching of
// Insert and IsConnected requests over one device-resident union-find state.
//
// Semantics (the batch-incremental correctness of ConnectIt's streaming
// appendix, with arrival order as the batch order): a query request sees
// exactly the insert requests that arrived before it.
//
// Two modes, by the server's union-find variant:
//
//  * Stamped (UF-Async with FindNaive, the default).  The parent array holds
//    64-bit words (insert stamp << 32 | parent).  Consecutive insert requests
//    with no query between them form an insert phase; phases are numbered
//    1, 2, ... in arrival order and every link a phase creates carries its
//    number.  Requests of one phase run concurrently on several HIP streams;
//    a phase starts after the previous one has completed.  A query that
//    arrives after phase t waits for phase t to complete and then follows
//    only links stamped <= t, so it runs concurrently with later insert
//    phases and still answers against exactly the inserts that arrived
//    before it: FindNaive never rewrites a link and a root's word changes
//    once, from "root" to a link stamped with a later phase, so the links
//    stamped <= t are exactly the forest that phases 1..t build when run
//    alone (each of them ran after the previous one and saw no later link).
//  * Barrier (every other variant, whose finds or splices rewrite links).
//    Consecutive requests of one type form a phase whose requests run
//    concurrently; at a change of type a barrier event orders the new phase
//    after the old one.
//
// Requests are admitted in arrival order when their device bytes fit in the
// memory budget and a slot is free, so new work starts while older work is
// still running.  The loop's state is bounded: a request is freed when it
// completes (its latency goes to a ring of recent completions, and to the
// caller's array for a trace replay), HIP events are recycled, and a phase
// only tracks its requests still in flight (a completed request needs no
// wait).
//
// Host side: the caller's buffers must stay valid until the request
// completes.  When they are pinned host memory mapped into the device's
// address space, the kernels read the pairs and write the answers in place
// (no pool bytes, no copies).  Otherwise the pairs are DMA'd into the pool
// on a copy stream of their own that no phase barrier holds up, and the
// answers are copied back.  Device side: a first-fit pool of the budget.
// Latency = completion (observed by polling the request's event) minus
// arrival, on the host's steady clock.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <unordered_map>
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
  size_t bytes = 0, off = 0;
  int stream = -1;
  hipEvent_t ev = nullptr;       // completion, on the request's stream
  hipEvent_t ev_copy = nullptr;  // payload on the device, on the copy stream
  uint8_t* out_host = nullptr;  // caller's result buffer (queries)
  const int32_t* a = nullptr;   // caller's payload (valid until completion)
  const int32_t* b = nullptr;
  double* latency_out = nullptr;  // trace replay: where the latency goes
  // mapped host memory: the kernels read the payload and write the answers
  // in place through these device addresses (no pool bytes, no copies)
  bool in_place = false;
  const int32_t* da = nullptr;
  const int32_t* db = nullptr;
  uint8_t* dout = nullptr;
  uint32_t phase = 0;             // stamped mode: the insert phases a query sees
};

// Completions kept for cc_server_request_info (the most recent ones).
constexpr int64_t kInfoRing = (int64_t)1 << 16;
struct Done {
  int64_t id = -1;
  double latency = 0.0;
};

// ---- stamped union-find (UF-Async, FindNaive) ------------------------------
// Word of vertex x: (stamp << 32) | parent; a root is (0 << 32) | x.
__device__ __forceinline__ uint64_t ldw(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x in the forest of the links stamped <= t (t = ~0u: every link).
__device__ __forceinline__ int32_t find_stamped(const uint64_t* W, int32_t x, uint32_t t) {
  while (true) {
    const uint64_t w = ldw(W + x);
    const int32_t p = (int32_t)(uint32_t)w;
    if (p == x || (uint32_t)(w >> 32) > t) return x;
    x = p;
  }
}

// Root of x over every link, for inserts, with path splitting where no
// query that can still run tells the difference.  A query of phase t
// follows exactly the links stamped <= t, so replacing x -> p (stamp s1)
// and p -> g (stamp s2) by x -> g stamped max(s1, s2) changes its answer
// only if min(s1, s2) <= t < max(s1, s2).  [qlo, qhi] spans the phases of
// the queries in flight when the insert was launched (qlo > qhi: none);
// queries launched later wait for this insert and see every link it can
// touch.  So x is re-linked when s1 == s2, or both stamps are <= qlo, or
// both are > qhi.
__device__ __forceinline__ int32_t find_stamped_split(uint64_t* W, int32_t x, uint32_t qlo, uint32_t qhi) {
  while (true) {
    const uint64_t w = ldw(W + x);
    const int32_t p = (int32_t)(uint32_t)w;
    if (p == x) return x;
    const uint64_t wp = ldw(W + p);
    const int32_t g = (int32_t)(uint32_t)wp;
    if (g != p) {
      const uint32_t s1 = (uint32_t)(w >> 32), s2 = (uint32_t)(wp >> 32);
      const uint32_t lo = s1 < s2 ? s1 : s2, hi = s1 < s2 ? s2 : s1;
      if (lo == hi || hi <= qlo || lo > qhi) {
        uint64_t expect = w;
        __hip_atomic_compare_exchange_strong(W + x, &expect, ((uint64_t)hi << 32) | (uint32_t)g, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    x = p;
  }
}

__global__ void k_stamped_init(int64_t n, uint64_t* W) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) W[i] = (uint64_t)i;
}

// UF-Async: find both roots; CAS the larger root's word from "root" to a link
// under the smaller one, stamped with the insert phase; retry on failure.
__global__ void k_stamped_insert(int64_t k, const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                                 uint64_t* W, uint32_t stamp, uint32_t qlo, uint32_t qhi, int64_t n, uint32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += stride) {
    const int32_t a = u[i], b = v[i];
    if (a < 0 || b < 0 || (int64_t)a >= n || (int64_t)b >= n) {
      bad = true;
      continue;
    }
    if (a == b) continue;
    while (true) {
      int32_t ra = find_stamped_split(W, a, qlo, qhi), rb = find_stamped_split(W, b, qlo, qhi);
      if (ra == rb) break;
      if (ra < rb) {
        const int32_t x = ra;
        ra = rb;
        rb = x;
      }
      uint64_t expect = (uint64_t)(uint32_t)ra;
      if (__hip_atomic_compare_exchange_strong(W + ra, &expect, ((uint64_t)stamp << 32) | (uint32_t)rb,
                                               __ATOMIC_RELAXED, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        break;
    }
  }
  if (bad) atomicOr(err, kErrBadId);
}

__global__ void k_stamped_query(int64_t q, const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                                uint8_t* __restrict__ out, const uint64_t* W, uint32_t stamp, int64_t n,
                                uint32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q; i += stride) {
    const int32_t x = a[i], y = b[i];
    if (x < 0 || y < 0 || (int64_t)x >= n || (int64_t)y >= n) {
      bad = true;
      out[i] = 0;
      continue;
    }
    out[i] = (x == y || find_stamped(W, x, stamp) == find_stamped(W, y, stamp)) ? 1 : 0;
  }
  if (bad) atomicOr(err, kErrBadId);
}

// Canonical labels of the whole forest (roots are tree minima: a link always
// goes from a larger root to a smaller one) and the number of components.
__global__ void k_stamped_labels(int64_t n, const uint64_t* W, int32_t* labels, long long* ncomp) {
  __shared__ long long red[256 / kWave];
  long long roots = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t r = find_stamped(W, (int32_t)v, ~0u);
    labels[v] = r;
    roots += (r == (int32_t)v);
  }
  roots = wave_sum(roots);
  if (lane_id() == 0) red[threadIdx.x / kWave] = roots;
  __syncthreads();
  if (threadIdx.x == 0 && ncomp) {
    long long t = 0;
    for (int i = 0; i < 256 / kWave; ++i) t += red[i];
    if (t) atomicAdd((unsigned long long*)ncomp, (unsigned long long)t);
  }
}

__global__ void k_server_zero(long long* p) { *p = 0; }

}  // namespace cc

struct cc_server {
  cc_ctx* ctx = nullptr;
  cc_stream* st = nullptr;      // barrier mode: the union-find state
  uint64_t* W = nullptr;        // stamped mode: stamped parent words
  uint32_t* err = nullptr;      // stamped mode: device error word
  bool stamped = false;
  int64_t n = 0;
  size_t budget = 0;
  int nstreams = 0;
  int max_inflight = 0;
  char* dpool = nullptr;
  cc::RangePool pool;
  std::vector<hipStream_t> streams;
  std::vector<int> stream_busy;  // requests in flight per stream
  hipStream_t copy_stream = nullptr;     // payload copies, in admission order
  hipStream_t barrier_stream = nullptr;
  std::vector<hipEvent_t> events_all;   // every event created; destroyed with the server
  std::vector<hipEvent_t> events_free;  // recycled, ready for a new record
  std::vector<hipEvent_t> barriers_old; // superseded barriers, recycled once complete
  std::deque<cc::Request*> pending;     // arrival order, not yet admitted
  std::vector<cc::Request*> inflight;
  std::unordered_map<int64_t, cc::Request*> live;  // submitted, not completed
  std::vector<cc::Done> done_ring;
  // phases
  int last_type = -1;                   // type of the last admitted request
  hipEvent_t barrier = nullptr;         // everything the next phase must wait for
  std::vector<cc::Request*> phase_open; // in-flight requests of the current phase (that a barrier must cover)
  uint32_t ins_phase = 0;               // stamped mode: insert phases started
  std::chrono::steady_clock::time_point t0;
  int64_t next_id = 0;
};

namespace cc {

static double now_s(const cc_server* s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

static hipEvent_t take_event(cc_server* s) {
  if (!s->events_free.empty()) {
    hipEvent_t e = s->events_free.back();
    s->events_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  s->events_all.push_back(e);
  return e;
}

// Superseded barriers are reused once they have completed: every wait that
// referred to them was enqueued before they were superseded.
static void recycle_barriers(cc_server* s) {
  for (size_t i = 0; i < s->barriers_old.size();) {
    if (hipEventQuery(s->barriers_old[i]) == hipSuccess) {
      s->events_free.push_back(s->barriers_old[i]);
      s->barriers_old[i] = s->barriers_old.back();
      s->barriers_old.pop_back();
    } else {
      ++i;
    }
  }
}

// Closes the current phase: a barrier event on the barrier stream after the
// previous barrier and every request of the phase still in flight (a
// completed request is already ordered before anything launched later).
static cc_status close_phase(cc_server* s) {
  if (s->barrier) CC_HIP(hipStreamWaitEvent(s->barrier_stream, s->barrier, 0));
  for (Request* r : s->phase_open) CC_HIP(hipStreamWaitEvent(s->barrier_stream, r->ev, 0));
  hipEvent_t b = take_event(s);
  if (!b) return fail(CC_EDEVICE, "cannot create an event");
  CC_HIP(hipEventRecord(b, s->barrier_stream));
  if (s->barrier) s->barriers_old.push_back(s->barrier);
  s->barrier = b;
  s->phase_open.clear();
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
  // Phase bookkeeping.  Barrier mode: every change of type closes the phase.
  // Stamped mode: only an insert phase is ever waited for, so only the change
  // insert -> query closes one, and a new insert phase opens after a query.
  bool track = true;
  if (s->stamped) {
    if (r->type == 1 && s->last_type == 0) {
      cc_status st = close_phase(s);
      if (st != CC_OK) return st;
    }
    if (r->type == 0 && s->last_type != 0) ++s->ins_phase;
    track = r->type == 0;
  } else if (r->type != s->last_type && s->last_type != -1) {
    cc_status st = close_phase(s);
    if (st != CC_OK) return st;
  }
  s->last_type = r->type;
  const int32_t* a = r->da;
  const int32_t* b = r->db;
  uint8_t* out = r->dout;
  if (!r->in_place) {
    // The payload goes over on the copy stream, which never waits for a
    // phase, so copies keep the link busy while earlier phases compute; the
    // request's stream waits for its copy and for the barrier.
    CC_HIP(hipMemcpyAsync(d, r->a, half, hipMemcpyHostToDevice, s->copy_stream));
    CC_HIP(hipMemcpyAsync(d + half, r->b, half, hipMemcpyHostToDevice, s->copy_stream));
    r->ev_copy = take_event(s);
    if (!r->ev_copy) return fail(CC_EDEVICE, "cannot create an event");
    CC_HIP(hipEventRecord(r->ev_copy, s->copy_stream));
    CC_HIP(hipStreamWaitEvent(hs, r->ev_copy, 0));
    a = (const int32_t*)d;
    b = (const int32_t*)(d + half);
    out = (uint8_t*)(d + pair_bytes);
  }
  if (s->barrier) CC_HIP(hipStreamWaitEvent(hs, s->barrier, 0));
  cc_status st = CC_OK;
  if (s->stamped) {
    const unsigned g = grid_for(r->k, 256, 8192);
    r->phase = s->ins_phase;
    if (r->type == 0) {
      // the phases of the queries in flight bound which links may be split
      uint32_t qlo = 0xffffffffu, qhi = 0;
      for (const Request* q : s->inflight)
        if (q->type == 1) {
          qlo = q->phase < qlo ? q->phase : qlo;
          qhi = q->phase > qhi ? q->phase : qhi;
        }
      hipLaunchKernelGGL(k_stamped_insert, dim3(g), dim3(256), 0, hs, r->k, a, b, s->W, s->ins_phase, qlo, qhi, s->n,
                         s->err);
    } else
      hipLaunchKernelGGL(k_stamped_query, dim3(g), dim3(256), 0, hs, r->k, a, b, out, (const uint64_t*)s->W,
                         s->ins_phase, s->n, s->err);
    CC_LAUNCH_CHECK();
  } else if (r->type == 0) {
    st = cc_insert_batch(s->st, r->k, a, b, hs);
  } else {
    st = cc_query_batch(s->st, r->k, a, b, out, hs);
  }
  if (st != CC_OK) return st;
  if (r->type == 1 && !r->in_place)
    CC_HIP(hipMemcpyAsync(r->out_host, out, (size_t)r->k, hipMemcpyDeviceToHost, hs));
  r->ev = take_event(s);
  if (!r->ev) return fail(CC_EDEVICE, "cannot create an event");
  CC_HIP(hipEventRecord(r->ev, hs));
  if (track) s->phase_open.push_back(r);
  s->inflight.push_back(r);
  return CC_OK;
}

// A request has completed: its memory, stream slot and event go back, its
// latency is recorded, and it is freed.
static void retire(cc_server* s, Request* r, double now) {
  const double lat = now - r->arrival;
  if (!r->in_place) s->pool.release(r->off, r->bytes);
  s->stream_busy[r->stream]--;
  auto it = std::find(s->phase_open.begin(), s->phase_open.end(), r);
  if (it != s->phase_open.end()) {
    *it = s->phase_open.back();
    s->phase_open.pop_back();
  }
  s->events_free.push_back(r->ev);
  if (r->ev_copy) s->events_free.push_back(r->ev_copy);  // complete: the request's stream waited for it
  if (r->latency_out) *r->latency_out = lat;
  Done& d = s->done_ring[(size_t)(r->id % kInfoRing)];
  d.id = r->id;
  d.latency = lat;
  s->live.erase(r->id);
  delete r;
}

}  // namespace cc

using namespace cc;

extern "C" {

cc_status cc_server_create(cc_ctx* ctx, int64_t n, const cc_variant* v, int64_t budget_bytes, int num_streams,
                           int max_inflight, cc_server** out) {
  if (!ctx || !out) return fail(CC_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 1 || n > 0x7fffffffLL) return fail(CC_EINVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
  if (budget_bytes < 4096) return fail(CC_EINVAL, "budget below 4 KiB");
  if (num_streams < 1 || num_streams > 16) return fail(CC_EINVAL, "num_streams must be in [1, 16]");
  if (max_inflight < 1 || max_inflight > 1024) return fail(CC_EINVAL, "max_inflight must be in [1, 1024]");
  if (v) {
    cc_status vs = check_variant(v, true);
    if (vs != CC_OK) return vs;
  }
  CC_HIP(hipSetDevice(ctx->device));
  cc_server* s = new cc_server();
  s->ctx = ctx;
  s->n = n;
  s->stamped = !v || (v->finish == CC_FIN_UF_ASYNC && v->find == CC_FIND_NAIVE);
  cc_status st = CC_OK;
  if (s->stamped) {
    if (hipMalloc((void**)&s->W, (size_t)n * 8) != hipSuccess || hipMalloc((void**)&s->err, 256) != hipSuccess)
      st = fail(CC_ENOMEM, "cannot allocate the stamped union-find state (%lld vertices)", (long long)n);
  } else {
    st = cc_stream_create(ctx, n, v, &s->st);
  }
  if (st == CC_OK && hipMalloc((void**)&s->dpool, (size_t)budget_bytes) != hipSuccess)
    st = fail(CC_ENOMEM, "cannot allocate a %lld-byte request pool", (long long)budget_bytes);
  if (st != CC_OK) {
    if (s->W) (void)hipFree(s->W);
    if (s->err) (void)hipFree(s->err);
    if (s->st) cc_stream_destroy(s->st);
    delete s;
    return st;
  }
  s->budget = (size_t)budget_bytes;
  s->nstreams = num_streams;
  s->max_inflight = max_inflight;
  s->pool.reset(s->budget);
  s->done_ring.assign((size_t)kInfoRing, Done{});
  s->streams.assign(num_streams, nullptr);
  s->stream_busy.assign(num_streams, 0);
  for (auto& x : s->streams) CC_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
  CC_HIP(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking));
  CC_HIP(hipStreamCreateWithFlags(&s->barrier_stream, hipStreamNonBlocking));
  if (s->stamped) {
    hipLaunchKernelGGL(k_stamped_init, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s->barrier_stream, n, s->W);
    CC_HIP(hipMemsetAsync(s->err, 0, 256, s->barrier_stream));
    CC_HIP(hipStreamSynchronize(s->barrier_stream));
  }
  s->t0 = std::chrono::steady_clock::now();
  *out = s;
  return CC_OK;
}

void cc_server_destroy(cc_server* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  for (auto* r : s->pending) delete r;
  for (auto* r : s->inflight) delete r;
  for (auto e : s->events_all) (void)hipEventDestroy(e);
  for (auto x : s->streams) (void)hipStreamDestroy(x);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  if (s->barrier_stream) (void)hipStreamDestroy(s->barrier_stream);
  if (s->dpool) (void)hipFree(s->dpool);
  if (s->W) (void)hipFree(s->W);
  if (s->err) (void)hipFree(s->err);
  if (s->st) cc_stream_destroy(s->st);
  delete s;
}

double cc_server_clock(cc_server* s) { return s ? now_s(s) : 0.0; }

int32_t cc_server_stamped(const cc_server* s) { return s && s->stamped ? 1 : 0; }

int64_t cc_server_event_count(const cc_server* s) { return s ? (int64_t)s->events_all.size() : -1; }

}  // extern "C"

namespace cc {

// Device address of a host range the GPU can read and write in place (host
// memory pinned and mapped into the device's address space, such as
// hipHostMalloc's), or nullptr.  Both ends of the range must map to the same
// allocation at the same distance, so the kernels never reach past it.
static void* mapped_host(const void* p, size_t bytes) {
  hipPointerAttribute_t a0{}, a1{};
  if (hipPointerGetAttributes(&a0, p) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a0.type != hipMemoryTypeHost || !a0.devicePointer) return nullptr;
  const char* last = (const char*)p + bytes - 1;
  if (hipPointerGetAttributes(&a1, last) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  if (a1.type != hipMemoryTypeHost || !a1.devicePointer ||
      (const char*)a1.devicePointer - (const char*)a0.devicePointer != (ptrdiff_t)(bytes - 1))
    return nullptr;
  return a0.devicePointer;
}

static cc_status submit(cc_server* s, int type, int64_t k, const int32_t* a, const int32_t* b, uint8_t* out,
                        double arrival, int64_t* id, double* latency_out = nullptr) {
  if (!s) return fail(CC_EINVAL, "server is NULL");
  if (k < 1) return fail(CC_EINVAL, "a request needs at least one pair");
  if (!a || !b || (type == 1 && !out)) return fail(CC_EINVAL, "NULL array");
  const int32_t* da = (const int32_t*)mapped_host(a, (size_t)k * 4);
  const int32_t* db = da ? (const int32_t*)mapped_host(b, (size_t)k * 4) : nullptr;
  uint8_t* dout = (db && type == 1) ? (uint8_t*)mapped_host(out, (size_t)k) : nullptr;
  const bool in_place = db && (type == 0 || dout);
  const size_t bytes = in_place ? 0 : (size_t)k * 8 + (type == 1 ? (size_t)k : 0);
  if (align256(bytes) > s->budget)
    return fail(CC_EBUSY, "request of %zu bytes can never fit the %zu-byte budget", bytes, s->budget);
  Request* r = new Request();
  r->id = s->next_id++;
  r->type = type;
  r->k = k;
  r->arrival = arrival >= 0 ? arrival : now_s(s);
  r->bytes = bytes;
  r->out_host = out;
  r->a = a;
  r->b = b;
  r->latency_out = latency_out;
  r->in_place = in_place;
  r->da = da;
  r->db = db;
  r->dout = dout;
  s->live[r->id] = r;
  s->pending.push_back(r);
  if (id) *id = r->id;
  return CC_OK;
}

// Retires finished requests, then admits pending ones in arrival order while
// memory and stream slots allow.
static cc_status progress_staged(cc_server* s) {
  for (size_t i = 0; i < s->inflight.size();) {
    Request* r = s->inflight[i];
    hipError_t q = hipEventQuery(r->ev);
    if (q == hipSuccess) {
      s->inflight[i] = s->inflight.back();
      s->inflight.pop_back();
      retire(s, r, now_s(s));
    } else if (q == hipErrorNotReady) {
      ++i;
    } else {
      return fail(CC_EDEVICE, "request event failed: %s", hipGetErrorString(q));
    }
  }
  recycle_barriers(s);
  while (!s->pending.empty() && (int)s->inflight.size() < s->max_inflight) {
    Request* r = s->pending.front();
    size_t off = 0;
    if (!r->in_place && !s->pool.alloc(r->bytes, &off)) break;
    r->off = off;
    s->pending.pop_front();
    cc_status st = launch(s, r);
    if (st != CC_OK) return st;
  }
  return CC_OK;
}

// Device error word of the server's state (reported once, then cleared).
static cc_status server_sync_status(cc_server* s) {
  if (!s->stamped) return cc_stream_sync_status(s->st);
  CC_HIP(hipDeviceSynchronize());
  uint32_t e = 0;
  CC_HIP(hipMemcpy(&e, s->err, 4, hipMemcpyDeviceToHost));
  if (e) {
    CC_HIP(hipMemset(s->err, 0, 4));
    return fail(CC_EDEVICE, "device error word 0x%x (1: id out of range)", e);
  }
  return CC_OK;
}

}  // namespace cc

extern "C" {

cc_status cc_server_submit_insert(cc_server* s, int64_t k, const int32_t* u, const int32_t* v, double arrival,
                                  int64_t* id) {
  return submit(s, 0, k, u, v, nullptr, arrival, id);
}

cc_status cc_server_submit_query(cc_server* s, int64_t q, const int32_t* a, const int32_t* b, uint8_t* out,
                                 double arrival, int64_t* id) {
  return submit(s, 1, q, a, b, out, arrival, id);
}

cc_status cc_server_poll(cc_server* s, int wait_all) {
  if (!s) return fail(CC_EINVAL, "server is NULL");
  do {
    cc_status st = progress_staged(s);
    if (st != CC_OK) return st;
  } while (wait_all && (!s->pending.empty() || !s->inflight.empty()));
  if (wait_all) return server_sync_status(s);
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
  for (int64_t i = 0; i < count; ++i) {
    while (now_s(s) - base < arrival_s[i]) {
      cc_status st = progress_staged(s);
      if (st != CC_OK) return st;
    }
    latency_s[i] = -1.0;
    cc_status st = submit(s, type[i] ? 1 : 0, len[i], a + start[i], b + start[i], type[i] ? out + start[i] : nullptr,
                          base + arrival_s[i], nullptr, &latency_s[i]);
    if (st != CC_OK) return st;
    st = progress_staged(s);
    if (st != CC_OK) return st;
  }
  return cc_server_poll(s, 1);
}

cc_status cc_server_request_info(cc_server* s, int64_t id, int* done, double* latency_s) {
  if (!s || id < 0 || id >= s->next_id) return fail(CC_EINVAL, "unknown request");
  if (s->live.count(id)) {
    if (done) *done = 0;
    if (latency_s) *latency_s = -1.0;
    return CC_OK;
  }
  const Done& d = s->done_ring[(size_t)(id % kInfoRing)];
  if (d.id != id) return fail(CC_EINVAL, "request %lld completed too long ago to be kept", (long long)id);
  if (done) *done = 1;
  if (latency_s) *latency_s = d.latency;
  return CC_OK;
}

cc_status cc_server_labels(cc_server* s, int32_t* labels_out, int64_t* num_components_dev, void* hip_stream) {
  if (!s) return fail(CC_EINVAL, "server is NULL");
  if (!labels_out) return fail(CC_EINVAL, "labels_out is NULL");
  cc_status st = cc_server_poll(s, 1);
  if (st != CC_OK) return st;
  if (!s->stamped) return cc_stream_labels(s->st, labels_out, num_components_dev, hip_stream);
  hipStream_t hs = (hipStream_t)hip_stream;
  if (num_components_dev) hipLaunchKernelGGL(k_server_zero, dim3(1), dim3(1), 0, hs, (long long*)num_components_dev);
  hipLaunchKernelGGL(k_stamped_labels, dim3(grid_for(s->n, 256, 4096)), dim3(256), 0, hs, s->n,
                     (const uint64_t*)s->W, labels_out, (long long*)num_components_dev);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

int64_t cc_server_pool_used(cc_server* s) { return s ? (int64_t)s->pool.used() : -1; }

}  // extern "C"
