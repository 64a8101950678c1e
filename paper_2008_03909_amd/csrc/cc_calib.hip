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
// Rows longer than a wave are reduced by the whole wave.
#include "cc_frontier.h"
#include "cc_static.h"

namespace cc {

__global__ void k_copy16(const int4* __restrict__ src, int4* __restrict__ dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

template <bool GATHER, typename I>
__global__ void k_edges_reduce(int64_t n, const I* __restrict__ off, const int32_t* __restrict__ adj,
                               const int32_t* __restrict__ vals, int32_t* __restrict__ out) {
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    int64_t b = 0, e = 0;
    if (v < n) {
      b = (int64_t)off[v];
      e = (int64_t)off[v + 1];
    }
    const bool big = (e - b) > kWave;
    int32_t acc = 0;
    uint64_t bm = __ballot(big);
    while (bm) {
      const int l = __ffsll((unsigned long long)bm) - 1;
      bm &= bm - 1;
      const int64_t bb = __shfl(b, l, kWave), eb = __shfl(e, l, kWave);
      int32_t part = 0;
      for (int64_t j = bb + lane; j < eb; j += kWave) {
        const int32_t w = adj[j];
        part += GATHER ? vals[w] : (w >= 0 ? 1 : 0);
      }
      part = wave_sum(part);
      if (lane == l) acc = part;
    }
    if (!big) {
      for (int64_t j = b; j < e; ++j) {
        const int32_t w = adj[j];
        acc += GATHER ? vals[w] : (w >= 0 ? 1 : 0);
      }
    }
    if (v < n) out[v] = acc;
  }
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

cc_status cc_calib_edges(int64_t n, const void* offsets, int offsets_are_64bit, const int32_t* adj,
                         const int32_t* vals, int32_t* out, void* hip_stream) {
  if (n < 1 || n > 0x7fffffffLL) return fail(CC_EINVAL, "bad n");
  if (!offsets || !out) return fail(CC_EINVAL, "NULL pointer");  // adj may be NULL when m == 0
  hipStream_t s = (hipStream_t)hip_stream;
  const unsigned g = grid_for(n, 256, 8192);
  if (offsets_are_64bit) {
    if (vals)
      hipLaunchKernelGGL((k_edges_reduce<true, int64_t>), dim3(g), dim3(256), 0, s, n, (const int64_t*)offsets, adj,
                         vals, out);
    else
      hipLaunchKernelGGL((k_edges_reduce<false, int64_t>), dim3(g), dim3(256), 0, s, n, (const int64_t*)offsets, adj,
                         vals, out);
  } else {
    if (vals)
      hipLaunchKernelGGL((k_edges_reduce<true, int32_t>), dim3(g), dim3(256), 0, s, n, (const int32_t*)offsets, adj,
                         vals, out);
    else
      hipLaunchKernelGGL((k_edges_reduce<false, int32_t>), dim3(g), dim3(256), 0, s, n, (const int32_t*)offsets, adj,
                         vals, out);
  }
  CC_LAUNCH_CHECK();
  return CC_OK;
}

}  // extern "C"
