// Calibration kernels: roofline anchors for the connectivity kernels.
//
//   copy          dst = src, 16-byte vectors (attainable HBM bandwidth)
//   map_edges     out[v] = number of adjacency entries read for v (the
//                 paper's MapEdges: map over vertices, reduce over incident
//                 edges with value 1 per edge)
//   gather_edges  out[v] = sum of vals[w] over v's neighbours w (the paper's
//                 GatherEdges: one indirect read per edge; its practical lower
//                 bound for any connectivity algorithm that always answers
//                 correctly, appendix "Comparison with MapEdges and
//                 GatherEdges")
// The adjacency array is cut into chunks of kCalibChunk consecutive
// entries, one block each, whatever rows they belong to, so every load is
// coalesced and every block has the same work (the CSR-stream scheme for
// sparse matrix-vector products).
#include "cc_frontier.h"
#include "cc_static.h"

namespace cc {

__global__ void k_copy16(const int4* __restrict__ src, int4* __restrict__ dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

constexpr int kCalibBlock = 256;
constexpr int kCalibPer = 8;                             // entries per lane
constexpr int64_t kCalibChunk = kCalibBlock * kCalibPer;  // entries per block
constexpr int kCalibRows = 2048;  // rows a chunk may span with its offsets staged in LDS

template <bool GATHER>
__device__ __forceinline__ int32_t edge_value(const int32_t* __restrict__ vals, int32_t w) {
  return GATHER ? vals[w] : (w >= 0 ? 1 : 0);
}

// One lane per row: crow[k] = the row holding entry k * kCalibChunk, for
// every chunk boundary inside the row, and crow[K] = the row holding the
// last entry; empty rows get their (zero) result here.
template <typename I>
__global__ void __launch_bounds__(kCalibBlock) k_edges_rows(int64_t n, int64_t m, const I* __restrict__ off,
                                                            int32_t* __restrict__ crow, int32_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += stride) {
    const int64_t b = (int64_t)off[r], e = (int64_t)off[r + 1];
    if (b == e) {
      out[r] = 0;
      continue;
    }
    for (int64_t k = (b + kCalibChunk - 1) / kCalibChunk; k * kCalibChunk < e; ++k) crow[k] = (int32_t)r;
    if (e == m) crow[(m + kCalibChunk - 1) / kCalibChunk] = (int32_t)r;
  }
}

// Block k reduces entries [k C, k C + C) (C = kCalibChunk): lane t loads
// entries 8t .. 8t + 7 of the chunk (two 16-byte loads when the array is
// aligned), finds the row of its first entry by binary search in the rows'
// offsets staged in LDS, and adds its values row by row into per-row LDS
// sums (one LDS atomic per row run).  The chunk then writes the rows that
// start in it; a row that started in an earlier chunk leaves its share in
// cont[k] for k_edges_carry.  A chunk that spans more than kCalibRows rows
// (runs of empty rows) walks them one lane per row instead.
template <bool GATHER, bool VEC, typename I>
__global__ void __launch_bounds__(kCalibBlock) k_edges_chunk(int64_t m, const I* __restrict__ off,
                                                             const int32_t* __restrict__ adj,
                                                             const int32_t* __restrict__ vals,
                                                             const int32_t* __restrict__ crow,
                                                             int32_t* __restrict__ out, int32_t* __restrict__ cont) {
  __shared__ int32_t rel[kCalibRows + 1];  // row offsets minus the chunk start, clamped to [-1, C + 1]
  __shared__ int32_t acc[kCalibRows];
  const int64_t k = blockIdx.x;
  const int64_t c0 = k * kCalibChunk;
  const int64_t len = (m - c0) < kCalibChunk ? (m - c0) : kCalibChunk;
  const int32_t r0 = crow[k];
  const int64_t nr = (int64_t)crow[k + 1] - r0 + 1;
  const int t = threadIdx.x;
  if (nr > kCalibRows) {
    for (int64_t i = t; i < nr; i += kCalibBlock) {
      const int64_t r = r0 + i;
      const int64_t b = (int64_t)off[r], e = (int64_t)off[r + 1];
      const int64_t lo = b > c0 ? b : c0, hi = e < c0 + len ? e : c0 + len;
      int32_t s = 0;
      for (int64_t j = lo; j < hi; ++j) s += edge_value<GATHER>(vals, adj[j]);
      if (b < e && b >= c0 && b < c0 + len) out[r] = s;
      else if (i == 0 && b < c0) cont[k] = s;
    }
    return;
  }
  for (int64_t i = t; i <= nr; i += kCalibBlock) {
    const int64_t x = (int64_t)off[r0 + i] - c0;
    rel[i] = (int32_t)(x < -1 ? -1 : x > kCalibChunk + 1 ? kCalibChunk + 1 : x);
    if (i < nr) acc[i] = 0;
  }
  __syncthreads();
  const int e0 = t * kCalibPer;
  if (e0 < len) {
    int32_t x[kCalibPer];
    if (VEC && e0 + kCalibPer <= len) {
#pragma unroll
      for (int q = 0; q < kCalibPer / 4; ++q) {
        const int4 a = *(const int4*)(adj + c0 + e0 + 4 * q);
        x[4 * q] = a.x, x[4 * q + 1] = a.y, x[4 * q + 2] = a.z, x[4 * q + 3] = a.w;
      }
    } else {
#pragma unroll
      for (int j = 0; j < kCalibPer; ++j) x[j] = e0 + j < len ? adj[c0 + e0 + j] : 0;
    }
    int32_t v[kCalibPer];
#pragma unroll
    for (int j = 0; j < kCalibPer; ++j) v[j] = e0 + j < len ? edge_value<GATHER>(vals, x[j]) : 0;
    // row of entry e0: the last i with rel[i] <= e0 (rows before it that
    // are empty share its offset and come first)
    int lo = 0, hi = (int)nr - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (rel[mid] <= e0) lo = mid;
      else hi = mid - 1;
    }
    int i = lo;
    int next = rel[i + 1];
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < kCalibPer; ++j) {
      if (e0 + j >= len) break;
      while (e0 + j >= next) {
        if (s) atomicAdd(acc + i, s);
        s = 0;
        ++i;
        next = rel[i + 1];
      }
      s += v[j];
    }
    if (s) atomicAdd(acc + i, s);
  }
  __syncthreads();
  for (int64_t i = t; i < nr; i += kCalibBlock) {
    const int32_t b = rel[i], e = rel[i + 1];
    if (b < e && b >= 0 && b < len) out[r0 + i] = acc[i];
    else if (i == 0 && b < 0) cont[k] = acc[0];
  }
}

// Adds the share of every row that continues across a chunk boundary.
template <typename I>
__global__ void k_edges_carry(int64_t K, const I* __restrict__ off, const int32_t* __restrict__ crow,
                              const int32_t* __restrict__ cont, int32_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < K; k += stride) {
    const int32_t r = crow[k];
    if ((int64_t)off[r] < k * kCalibChunk) atomicAdd(out + r, cont[k]);
  }
}

template <bool GATHER, typename I>
static void launch_edges(int64_t n, int64_t m, const I* off, const int32_t* adj, const int32_t* vals, int32_t* out,
                         char* w, hipStream_t s) {
  const int64_t K = (m + kCalibChunk - 1) / kCalibChunk;
  int32_t* crow = (int32_t*)w;
  int32_t* cont = (int32_t*)(w + align256((size_t)(K + 1) * 4));
  hipLaunchKernelGGL((k_edges_rows<I>), dim3(grid_for(n, kCalibBlock, 1 << 16)), dim3(kCalibBlock), 0, s, n, m, off,
                     crow, out);
  if (K == 0) return;
  if (((uintptr_t)adj & 15u) == 0)
    hipLaunchKernelGGL((k_edges_chunk<GATHER, true, I>), dim3((unsigned)K), dim3(kCalibBlock), 0, s, m, off, adj,
                       vals, (const int32_t*)crow, out, cont);
  else
    hipLaunchKernelGGL((k_edges_chunk<GATHER, false, I>), dim3((unsigned)K), dim3(kCalibBlock), 0, s, m, off, adj,
                       vals, (const int32_t*)crow, out, cont);
  if (K > 1)
    hipLaunchKernelGGL((k_edges_carry<I>), dim3(grid_for(K, kCalibBlock, 1024)), dim3(kCalibBlock), 0, s, K, off,
                       (const int32_t*)crow, (const int32_t*)cont, out);
}

}  // namespace cc

using namespace cc;

extern "C" {

cc_status cc_calib_copy(const void* src, void* dst, size_t bytes, void* hip_stream) {
  if (!src || !dst) return fail(CC_EINVAL, "NULL pointer");
  if ((bytes & 15u) || ((uintptr_t)src & 15u) || ((uintptr_t)dst & 15u))
    return fail(CC_EINVAL, "copy needs 16-byte aligned pointers and a multiple of 16 bytes");
  const int64_t count = (int64_t)(bytes / 16);
  if (count == 0) return CC_OK;
  hipLaunchKernelGGL(k_copy16, dim3(grid_for(count, 256, 8192)), dim3(256), 0, (hipStream_t)hip_stream,
                     (const int4*)src, (int4*)dst, count);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

cc_status cc_calib_workspace_bytes(int64_t m, size_t* bytes) {
  if (!bytes || m < 0) return fail(CC_EINVAL, "bad argument");
  // the row of every chunk boundary (and of the last entry), then each
  // chunk's share of a row that started before it
  const size_t K = (size_t)((m + kCalibChunk - 1) / kCalibChunk);
  *bytes = align256((K + 1) * 4) + align256((K + 1) * 4);
  return CC_OK;
}

cc_status cc_calib_edges(int64_t n, int64_t m, const void* offsets, int offsets_are_64bit, const int32_t* adj,
                         const int32_t* vals, int32_t* out, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (n < 1 || n > 0x7fffffffLL || m < 0) return fail(CC_EINVAL, "bad n or m");
  if (!offsets || !out) return fail(CC_EINVAL, "NULL pointer");  // adj may be NULL when m == 0
  size_t need = 0;
  cc_calib_workspace_bytes(m, &need);
  if (!workspace || ws_bytes < need) return fail(CC_ENOMEM, "workspace smaller than %zu bytes", need);
  hipStream_t s = (hipStream_t)hip_stream;
  char* w = (char*)workspace;
  if (offsets_are_64bit) {
    if (vals) launch_edges<true>(n, m, (const int64_t*)offsets, adj, vals, out, w, s);
    else launch_edges<false>(n, m, (const int64_t*)offsets, adj, vals, out, w, s);
  } else {
    if (vals) launch_edges<true>(n, m, (const int32_t*)offsets, adj, vals, out, w, s);
    else launch_edges<false>(n, m, (const int32_t*)offsets, adj, vals, out, w, s);
  }
  CC_LAUNCH_CHECK();
  return CC_OK;
}

}  // extern "C"
