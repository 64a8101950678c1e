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
                               const int32_t* __restrict__ vals, int32_t* __restrict__ out, int32_t* heavy,
                               int32_t* hcount) {
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    int64_t b = 0, e = 0;
    if (v < n) {
      b = (int64_t)off[v];
      e = (int64_t)off[v + 1];
    }
    const bool heavy_row = (e - b) > kHeavyFrontier;
    wave_append(heavy_row, (int32_t)v, heavy, (uint32_t*)hcount);
    if (heavy_row) e = b;  // reduced by k_edges_heavy
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

// Heavy rows: edges spread over the grid; per-vertex partial sums are added
// once per run of equal owners within a wave.
template <bool GATHER, typename I>
__global__ void k_edges_heavy(const int32_t* __restrict__ heavy, const int32_t* hcount,
                              const long long* __restrict__ hp, const I* __restrict__ off,
                              const int32_t* __restrict__ adj, const int32_t* __restrict__ vals,
                              int32_t* __restrict__ out) {
  const int64_t c = *hcount;
  if (c == 0) return;
  const long long T = hp[c];
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (long long base = blockIdx.x * (int64_t)blockDim.x; base < T; base += stride) {
    const long long e = base + threadIdx.x;
    int32_t u = -1, x = 0;
    const long long e0 = base + (threadIdx.x / kWave) * kWave;
    if (e < T) {
      const int64_t i = heavy_owner_tile(hp, c, e0, e);
      u = heavy[i];
      const int32_t w = adj[(int64_t)off[u] + (e - hp[i])];
      x = GATHER ? vals[w] : (w >= 0 ? 1 : 0);
    }
    uint64_t act = __ballot(u >= 0);
    while (act) {
      const int leader = __ffsll((unsigned long long)act) - 1;
      const int32_t lu = __shfl(u, leader, kWave);
      const bool mine = u == lu && u >= 0;
      const int32_t part = wave_sum(mine ? x : 0);
      if (lane == leader) atomicAdd(out + lu, part);
      act &= ~__ballot(mine);
      if (mine) u = -1;
    }
  }
}

__global__ void k_zero_i32(int32_t* p) { *p = 0; }

template <bool GATHER, typename I>
static void launch_edges(int64_t n, const I* off, const int32_t* adj, const int32_t* vals, int32_t* out, char* w,
                         size_t hcap, hipStream_t s) {
  int32_t* hcount = (int32_t*)w;
  int32_t* heavy = (int32_t*)(w + 256);
  long long* hp = (long long*)(w + 256 + align256(hcap * 4));
  long long* tsum = (long long*)(w + 256 + align256(hcap * 4) + align256((hcap + 1) * 8));
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(1), 0, s, hcount);
  hipLaunchKernelGGL((k_edges_reduce<GATHER, I>), dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, off, adj, vals,
                     out, heavy, hcount);
  heavy_prefix<I>(s, heavy, (const int32_t*)hcount, (int64_t)hcap, off, tsum, hp);
  hipLaunchKernelGGL((k_edges_heavy<GATHER, I>), dim3(2048), dim3(256), 0, s, (const int32_t*)heavy,
                     (const int32_t*)hcount, (const long long*)hp, off, adj, vals, out);
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
  const size_t hcap = heavy_cap(m);
  *bytes = 256 + align256(hcap * 4) + align256((hcap + 1) * 8) + align256((hcap / kHpTile + 3) * 8);
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
  const size_t hcap = heavy_cap(m);
  char* w = (char*)workspace;
  if (offsets_are_64bit) {
    if (vals) launch_edges<true>(n, (const int64_t*)offsets, adj, vals, out, w, hcap, s);
    else launch_edges<false>(n, (const int64_t*)offsets, adj, vals, out, w, hcap, s);
  } else {
    if (vals) launch_edges<true>(n, (const int32_t*)offsets, adj, vals, out, w, hcap, s);
    else launch_edges<false>(n, (const int32_t*)offsets, adj, vals, out, w, hcap, s);
  }
  CC_LAUNCH_CHECK();
  return CC_OK;
}

}  // extern "C"
