// Batch-incremental connectivity (ConnectIt Section 3.4 "Streaming";
// appendix "ConnectIt: Streaming").
//
// The stream keeps a device-resident parent array.  The finish decides how
// a batch runs, after the paper's three types of streaming algorithms:
//  * type 1 -- UF-Async, UF-Early, UF-Hooks (any find) and UF-Rem-CAS with
//    SplitAtomicOne or HalveAtomicOne: unions and finds are linearizable together, so a mixed
//    batch (cc_process_batch) runs its inserts and queries concurrently in
//    one kernel; a query is Jayanti and Tarjan's SameSet (find both roots;
//    equal: connected; else, if the first root is still a root, not
//    connected, linearized when the second find returned; else retry);
//  * type 2 -- Shiloach-Vishkin and the root-based Liu-Tarjan variants:
//    inserts are processed as a batch, in synchronous rounds over the
//    batch's edges until nothing changes, then the queries run;
//  * type 3 -- UF-Rem-CAS with SpliceAtomic: phase-concurrent, the batch's
//    inserts run concurrently, then (after a barrier) its queries.
// insert_batch / query_batch are the pure batches.  Calls on one stream are
// ordered by the HIP stream they are enqueued on, so a batch sees exactly
// the batches enqueued before it.
#include <algorithm>
#include <cstring>

#include "cc_device.h"
#include "cc_frontier.h"
#include "cc_static.h"

struct cc_stream {
  cc_ctx* ctx = nullptr;
  int64_t n = 0;
  cc_variant v{};
  int type = 1;                       // streaming type (1, 2 or 3) of the finish
  int32_t* P = nullptr;
  uint32_t* err = nullptr;
  int32_t* H = nullptr;               // UF-Hooks only: the claim array (-1 = unclaimed)
  // type 2 only: round snapshot and the batch's edge list (grown on demand)
  int32_t* Q = nullptr;
  int32_t* eu = nullptr;
  int32_t* ev = nullptr;
  unsigned long long* ecnt = nullptr;
  int64_t ecap = 0;
  int32_t last_rounds = 0;
};

namespace cc {

__global__ void k_stream_init(int64_t n, int32_t* P) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) P[i] = (int32_t)i;
}

template <int ALG, int SPLICE, int FIND>
__global__ void k_stream_insert(int64_t k, const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                                int32_t* P, int32_t* H, int64_t n, uint32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += stride) {
    const int32_t a = u[i], b = v[i];
    if (a < 0 || b < 0 || (int64_t)a >= n || (int64_t)b >= n) {
      bad = true;
      continue;
    }
    if (a != b) unite<ALG, SPLICE, FIND>(P, a, b, H);
  }
  if (bad) atomicOr(err, kErrBadId);
}

template <int FIND>
__global__ void k_stream_query(int64_t q, const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                               uint8_t* __restrict__ out, int32_t* P, int64_t n, uint32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q; i += stride) {
    const int32_t x = a[i], y = b[i];
    if (x < 0 || y < 0 || (int64_t)x >= n || (int64_t)y >= n) {
      bad = true;
      out[i] = 0;
      continue;
    }
    out[i] = (x == y || find<FIND>(P, x) == find<FIND>(P, y)) ? 1 : 0;
  }
  if (bad) atomicOr(err, kErrBadId);
}

// Jayanti-Tarjan SameSet: linearizable against concurrent unions that link
// roots only.  If ra is still a root after rb was found, ra and rb were
// both roots when rb was found, so x and y were apart at that moment.
// For UF-Hooks (H non-null) a root is one that is unclaimed in H, and the
// finds follow claims (a claim is the union's linearization point).
template <int FIND>
__device__ __forceinline__ bool same_set(int32_t* P, const int32_t* H, int32_t x, int32_t y) {
  if (x == y) return true;
  while (true) {
    const int32_t ra = H ? find_hooks<FIND>(P, H, x) : find<FIND>(P, x);
    const int32_t rb = H ? find_hooks<FIND>(P, H, y) : find<FIND>(P, y);
    if (ra == rb) return true;
    if (H ? ld(H + ra) < 0 : ld(P + ra) == ra) return false;
  }
}

// A mixed batch.  kind[i] == 0: Insert(u[i], v[i]); otherwise
// IsConnected(u[i], v[i]) -> out[i] (out[i] = 0 for inserts).  PHASE -1:
// both kinds in one pass (type 1); 0: inserts only; 1: queries only.
template <int ALG, int SPLICE, int FIND, int PHASE>
__global__ void k_stream_mixed(int64_t k, const uint8_t* __restrict__ kind, const int32_t* __restrict__ u,
                               const int32_t* __restrict__ v, uint8_t* __restrict__ out, int32_t* P, int32_t* H,
                               int64_t n, uint32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += stride) {
    const bool query = kind[i] != 0;
    if ((PHASE == 0 && query) || (PHASE == 1 && !query)) continue;
    const int32_t a = u[i], b = v[i];
    if (a < 0 || b < 0 || (int64_t)a >= n || (int64_t)b >= n) {
      bad = true;  // each operation is handled in exactly one phase
      out[i] = 0;
      continue;
    }
    if (query) {
      out[i] = same_set<FIND>(P, ALG == 3 ? H : nullptr, a, b) ? 1 : 0;
    } else {
      out[i] = 0;
      if (a != b) unite<ALG, SPLICE, FIND>(P, a, b, H);
    }
  }
  if (bad) atomicOr(err, kErrBadId);
}

// Inserts of a batch as an edge list for the round-based finishes: entry i
// is (u[i], v[i]) if it is a valid insert with u != v, else dead (-1).
__global__ void k_stream_edges(int64_t k, const uint8_t* __restrict__ kind, const int32_t* __restrict__ u,
                               const int32_t* __restrict__ v, int32_t* __restrict__ eu, int32_t* __restrict__ ev,
                               unsigned long long* ecnt, int64_t n, uint32_t* err, uint8_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *ecnt = (unsigned long long)k;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += stride) {
    const bool query = kind && kind[i] != 0;
    const int32_t a = u[i], b = v[i];
    const bool valid = a >= 0 && b >= 0 && (int64_t)a < n && (int64_t)b < n;
    if (!query && !valid) bad = true;
    eu[i] = (!query && valid && a != b) ? a : -1;
    ev[i] = b;
    if (out && !query) out[i] = 0;
  }
  if (bad) atomicOr(err, kErrBadId);
}

__global__ void k_stream_labels(int64_t n, int32_t* P, int32_t* labels, long long* ncomp) {
  __shared__ long long red[256 / kWave];
  long long roots = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t r = find_naive(P, (int32_t)v);
    labels[v] = r;
    roots += (r == (int32_t)v);
  }
  roots = wave_sum(roots);
  if (lane_id() == 0) red[threadIdx.x / kWave] = roots;
  __syncthreads();
  if (threadIdx.x == 0 && ncomp) {
    for (int w = 1; w < 256 / kWave; ++w) roots += red[w];
    if (roots) add64(ncomp, roots);
  }
}

__global__ void k_zero_i64(long long* p) { *p = 0; }

template <int ALG, int SPLICE, int FIND>
static void launch_insert(cc_stream* s, int64_t k, const int32_t* u, const int32_t* v, hipStream_t st) {
  hipLaunchKernelGGL((k_stream_insert<ALG, SPLICE, FIND>), dim3(grid_for(k, 256, 8192)), dim3(256), 0, st, k, u, v,
                     s->P, s->H, s->n, s->err);
}

template <int ALG, int SPLICE, int FIND, int PHASE>
static void launch_mixed(cc_stream* s, int64_t k, const uint8_t* kind, const int32_t* u, const int32_t* v,
                         uint8_t* out, hipStream_t st) {
  hipLaunchKernelGGL((k_stream_mixed<ALG, SPLICE, FIND, PHASE>), dim3(grid_for(k, 256, 8192)), dim3(256), 0, st, k,
                     kind, u, v, out, s->P, s->H, s->n, s->err);
}

// Dispatch of a mixed batch over the union-find variants (types 1 and 3).
template <int PHASE>
static void mixed_uf(cc_stream* s, int64_t k, const uint8_t* kind, const int32_t* u, const int32_t* v, uint8_t* out,
                     hipStream_t st) {
  const cc_variant& x = s->v;
#define FINDS(ALG)                                                       \
  {                                                                      \
    if (x.find == 0) launch_mixed<ALG, 0, 0, PHASE>(s, k, kind, u, v, out, st);      \
    else if (x.find == 1) launch_mixed<ALG, 0, 1, PHASE>(s, k, kind, u, v, out, st); \
    else if (x.find == 2) launch_mixed<ALG, 0, 2, PHASE>(s, k, kind, u, v, out, st); \
    else launch_mixed<ALG, 0, 3, PHASE>(s, k, kind, u, v, out, st);                 \
    return;                                                              \
  }
  if (x.finish == CC_FIN_UF_ASYNC) FINDS(1)
  if (x.finish == CC_FIN_UF_EARLY) FINDS(2)
  if (x.finish == CC_FIN_UF_HOOKS) FINDS(3)
#undef FINDS
#define REM(SPL, FND) \
  if (x.splice == SPL && x.find == FND) return launch_mixed<0, SPL, FND, PHASE>(s, k, kind, u, v, out, st);
  REM(0, 0) REM(0, 1) REM(0, 2) REM(1, 0) REM(1, 1) REM(1, 2) REM(2, 0) REM(2, 1) REM(2, 2)
#undef REM
}

static int stream_type(const cc_variant& v) {
  if (v.finish == CC_FIN_SV || v.finish == CC_FIN_LT) return 2;
  if (v.finish == CC_FIN_UF_REM_CAS && v.splice == CC_SPLICE_ATOMIC) return 3;
  return 1;
}

// Type 2: the batch's inserts as an edge list, then rounds until no change.
// The edge list has a fixed capacity, allocated with the stream; a larger
// batch is inserted as consecutive parts of that size, each run to its
// fixed point (the connectivity after all parts is that of the whole batch,
// union being associative), so an insert never allocates or waits for
// memory.
constexpr int64_t kType2EdgeCap = (int64_t)1 << 22;

static cc_status round_inserts(cc_stream* s, int64_t k, const uint8_t* kind, const int32_t* u, const int32_t* v,
                               uint8_t* out, hipStream_t st) {
  for (int64_t c0 = 0; c0 < k; c0 += s->ecap) {
    const int64_t kc = std::min<int64_t>(s->ecap, k - c0);
    hipLaunchKernelGGL(k_stream_edges, dim3(grid_for(kc, 256, 8192)), dim3(256), 0, st, kc,
                       kind ? kind + c0 : nullptr, u + c0, v + c0, s->eu, s->ev, s->ecnt, s->n, s->err,
                       out ? out + c0 : nullptr);
    CC_LAUNCH_CHECK();
    int32_t rounds = 0;
    cc_status r = edge_list_rounds(s->ctx, st, s->v, s->n, s->P, s->Q, s->eu, s->ev, s->ecnt, kc, &rounds);
    if (r != CC_OK) return r;
    s->last_rounds = c0 == 0 ? rounds : s->last_rounds + rounds;
  }
  return CC_OK;
}

}  // namespace cc

using namespace cc;

extern "C" {

cc_status cc_stream_create(cc_ctx* ctx, int64_t n, const cc_variant* v, cc_stream** out) {
  if (!ctx || !out) return fail(CC_EINVAL, "NULL argument");
  *out = nullptr;
  if (n < 1 || n > 0x7fffffffLL) return fail(CC_EINVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
  cc_variant dv;
  if (!v) {
    cc_default_variant(&dv);
    dv.finish = CC_FIN_UF_ASYNC;
    dv.find = CC_FIND_NAIVE;
    v = &dv;
  }
  cc_status st = check_variant(v, true);
  if (st != CC_OK) return st;
  CC_HIP(hipSetDevice(ctx->device));
  cc_stream* s = new cc_stream();
  s->ctx = ctx;
  s->n = n;
  s->v = *v;
  s->type = stream_type(*v);
  bool ok = hipMalloc((void**)&s->P, (size_t)n * 4) == hipSuccess && hipMalloc((void**)&s->err, 256) == hipSuccess;
  if (ok && s->type == 2) {
    ok = hipMalloc((void**)&s->Q, (size_t)n * 4) == hipSuccess && hipMalloc((void**)&s->ecnt, 256) == hipSuccess &&
         hipMalloc((void**)&s->eu, (size_t)kType2EdgeCap * 4) == hipSuccess &&
         hipMalloc((void**)&s->ev, (size_t)kType2EdgeCap * 4) == hipSuccess;
    s->ecap = kType2EdgeCap;
  }
  if (ok && v->finish == CC_FIN_UF_HOOKS) {
    ok = hipMalloc((void**)&s->H, (size_t)n * 4) == hipSuccess;
    if (ok) ok = hipMemset(s->H, 0xff, (size_t)n * 4) == hipSuccess;
  }
  if (!ok) {
    for (void* p : {(void*)s->P, (void*)s->err, (void*)s->H, (void*)s->Q, (void*)s->ecnt, (void*)s->eu, (void*)s->ev})
      if (p) (void)hipFree(p);
    delete s;
    return fail(CC_ENOMEM, "cannot allocate the stream state (%lld vertices)", (long long)n);
  }
  hipLaunchKernelGGL(k_stream_init, dim3(grid_for(n, 256, 4096)), dim3(256), 0, (hipStream_t)0, n, s->P);
  if (hipMemset(s->err, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    cc_stream_destroy(s);
    return fail(CC_EDEVICE, "stream initialisation failed");
  }
  *out = s;
  return CC_OK;
}

void cc_stream_destroy(cc_stream* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();  // teardown: errors have nowhere to go
  for (void* p : {(void*)s->P, (void*)s->err, (void*)s->H, (void*)s->Q, (void*)s->eu, (void*)s->ev, (void*)s->ecnt})
    if (p) (void)hipFree(p);
  delete s;
}

cc_status cc_stream_init_csr(cc_stream* s, int64_t m, const void* offsets, int offsets_are_64bit,
                             const int32_t* adj, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!s) return fail(CC_EINVAL, "stream is NULL");
  return cc_connectivity_csr(s->ctx, s->n, m, offsets, offsets_are_64bit, adj, &s->v, workspace, ws_bytes, s->P,
                             nullptr, hip_stream);
}

cc_status cc_insert_batch(cc_stream* s, int64_t k, const int32_t* u, const int32_t* v, void* hip_stream) {
  if (!s) return fail(CC_EINVAL, "stream is NULL");
  if (k < 0) return fail(CC_EINVAL, "k < 0");
  if (k == 0) return CC_OK;
  if (!u || !v) return fail(CC_EINVAL, "NULL pair array");
  hipStream_t st = (hipStream_t)hip_stream;
  if (s->type == 2) return round_inserts(s, k, nullptr, u, v, nullptr, st);
  const cc_variant& x = s->v;
#define FINDS(ALG)                                        \
  {                                                       \
    if (x.find == 0) launch_insert<ALG, 0, 0>(s, k, u, v, st);      \
    else if (x.find == 1) launch_insert<ALG, 0, 1>(s, k, u, v, st); \
    else if (x.find == 2) launch_insert<ALG, 0, 2>(s, k, u, v, st); \
    else launch_insert<ALG, 0, 3>(s, k, u, v, st);                 \
  }
  if (x.finish == CC_FIN_UF_ASYNC) FINDS(1)
  else if (x.finish == CC_FIN_UF_EARLY) FINDS(2)
  else if (x.finish == CC_FIN_UF_HOOKS) FINDS(3)
#undef FINDS
  else {
#define REM(SPL, FND) \
  else if (x.splice == SPL && x.find == FND) launch_insert<0, SPL, FND>(s, k, u, v, st);
    if (false) {
    }
    REM(0, 0) REM(0, 1) REM(0, 2) REM(1, 0) REM(1, 1) REM(1, 2) REM(2, 0) REM(2, 1) REM(2, 2)
#undef REM
  }
  CC_LAUNCH_CHECK();
  return CC_OK;
}

cc_status cc_query_batch(cc_stream* s, int64_t q, const int32_t* a, const int32_t* b, uint8_t* out,
                         void* hip_stream) {
  if (!s) return fail(CC_EINVAL, "stream is NULL");
  if (q < 0) return fail(CC_EINVAL, "q < 0");
  if (q == 0) return CC_OK;
  if (!a || !b || !out) return fail(CC_EINVAL, "NULL array");
  hipStream_t st = (hipStream_t)hip_stream;
  const unsigned g = grid_for(q, 256, 8192);
  // Finds that compress are safe here: queries never overlap inserts on one stream.
  switch (s->v.find) {
    case CC_FIND_ATOMIC_SPLIT:
      hipLaunchKernelGGL(k_stream_query<kFindSplit>, dim3(g), dim3(256), 0, st, q, a, b, out, s->P, s->n, s->err);
      break;
    case CC_FIND_ATOMIC_HALVE:
      hipLaunchKernelGGL(k_stream_query<kFindHalve>, dim3(g), dim3(256), 0, st, q, a, b, out, s->P, s->n, s->err);
      break;
    case CC_FIND_COMPRESS:
      hipLaunchKernelGGL(k_stream_query<kFindCompress>, dim3(g), dim3(256), 0, st, q, a, b, out, s->P, s->n,
                         s->err);
      break;
    default:
      hipLaunchKernelGGL(k_stream_query<kFindNaive>, dim3(g), dim3(256), 0, st, q, a, b, out, s->P, s->n, s->err);
  }
  CC_LAUNCH_CHECK();
  return CC_OK;
}

cc_status cc_process_batch(cc_stream* s, int64_t k, const uint8_t* kind, const int32_t* u, const int32_t* v,
                           uint8_t* out, void* hip_stream) {
  if (!s) return fail(CC_EINVAL, "stream is NULL");
  if (k < 0) return fail(CC_EINVAL, "k < 0");
  if (k == 0) return CC_OK;
  if (!kind || !u || !v || !out) return fail(CC_EINVAL, "NULL array");
  hipStream_t st = (hipStream_t)hip_stream;
  if (s->type == 1) {
    mixed_uf<-1>(s, k, kind, u, v, out, st);
  } else if (s->type == 3) {
    mixed_uf<0>(s, k, kind, u, v, out, st);
    mixed_uf<1>(s, k, kind, u, v, out, st);
  } else {
    cc_status r = round_inserts(s, k, kind, u, v, out, st);
    if (r != CC_OK) return r;
    // queries after the rounds: P is a min-based forest, naive finds
    hipLaunchKernelGGL((k_stream_mixed<1, 0, 0, 1>), dim3(grid_for(k, 256, 8192)), dim3(256), 0, st, k, kind, u, v,
                       out, s->P, (int32_t*)nullptr, s->n, s->err);
  }
  CC_LAUNCH_CHECK();
  return CC_OK;
}

int32_t cc_stream_type(const cc_stream* s) { return s ? s->type : 0; }

cc_status cc_stream_labels(cc_stream* s, int32_t* labels_out, int64_t* num_components_dev, void* hip_stream) {
  if (!s || !labels_out) return fail(CC_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)hip_stream;
  if (num_components_dev) hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, st, (long long*)num_components_dev);
  hipLaunchKernelGGL(k_stream_labels, dim3(grid_for(s->n, 256, 4096)), dim3(256), 0, st, s->n, s->P, labels_out,
                     (long long*)num_components_dev);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

cc_status cc_stream_sync_status(cc_stream* s) {
  if (!s) return fail(CC_EINVAL, "stream is NULL");
  CC_HIP(hipDeviceSynchronize());
  uint32_t e = 0;
  CC_HIP(hipMemcpy(&e, s->err, 4, hipMemcpyDeviceToHost));
  if (e) {
    CC_HIP(hipMemset(s->err, 0, 4));
    return fail(CC_EDEVICE, "device error word 0x%x: a pair id was outside [0, n)", e);
  }
  return CC_OK;
}

}  // extern "C"
