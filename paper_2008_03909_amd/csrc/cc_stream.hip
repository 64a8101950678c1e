// Batch-incremental connectivity (ConnectIt Section 3.4; appendix
// "ConnectIt: Streaming").
//
// The stream keeps a device-resident parent array.  insert_batch applies
// Union(u, v) for every pair of the batch concurrently; query_batch answers
// IsConnected(a, b) as find(a) == find(b).  Calls on one stream are ordered by
// the HIP stream they are enqueued on, so a query batch sees exactly the
// insert batches enqueued before it -- the batch-incremental correctness of
// the paper for all union-find types, including Rem's algorithm with the
// splice rule, whose inserts and finds must not overlap (phase-concurrent).
#include <cstring>

#include "cc_device.h"
#include "cc_frontier.h"
#include "cc_static.h"

struct cc_stream {
  cc_ctx* ctx = nullptr;
  int64_t n = 0;
  cc_variant v{};
  int32_t* P = nullptr;
  uint32_t* err = nullptr;
};

namespace cc {

__global__ void k_stream_init(int64_t n, int32_t* P) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) P[i] = (int32_t)i;
}

template <int ALG, int SPLICE, int FIND>
__global__ void k_stream_insert(int64_t k, const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                                int32_t* P, int64_t n, uint32_t* err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += stride) {
    const int32_t a = u[i], b = v[i];
    if (a < 0 || b < 0 || (int64_t)a >= n || (int64_t)b >= n) {
      bad = true;
      continue;
    }
    if (a != b) unite<ALG, SPLICE, FIND>(P, a, b);
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
                     s->P, s->n, s->err);
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
  if (hipMalloc((void**)&s->P, (size_t)n * 4) != hipSuccess || hipMalloc((void**)&s->err, 256) != hipSuccess) {
    if (s->P) hipFree(s->P);
    delete s;
    return fail(CC_ENOMEM, "cannot allocate the stream state (%lld vertices)", (long long)n);
  }
  hipLaunchKernelGGL(k_stream_init, dim3(grid_for(n, 256, 4096)), dim3(256), 0, (hipStream_t)0, n, s->P);
  hipMemset(s->err, 0, 256);
  if (hipDeviceSynchronize() != hipSuccess) {
    hipFree(s->P);
    hipFree(s->err);
    delete s;
    return fail(CC_EDEVICE, "stream initialisation failed");
  }
  *out = s;
  return CC_OK;
}

void cc_stream_destroy(cc_stream* s) {
  if (!s) return;
  hipDeviceSynchronize();
  hipFree(s->P);
  hipFree(s->err);
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
  const cc_variant& x = s->v;
  if (x.finish == CC_FIN_UF_ASYNC) {
    if (x.find == 0) launch_insert<1, 0, 0>(s, k, u, v, st);
    else if (x.find == 1) launch_insert<1, 0, 1>(s, k, u, v, st);
    else if (x.find == 2) launch_insert<1, 0, 2>(s, k, u, v, st);
    else launch_insert<1, 0, 3>(s, k, u, v, st);
  } else {
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
