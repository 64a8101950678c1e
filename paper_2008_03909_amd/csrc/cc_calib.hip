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
// Rows are binned by length, the same way the connectivity kernels bin
// their candidate vertices: a lane reduces a row of up to 32 entries, a wave
// one of up to 4096, and longer rows are cut into edge chunks spread over
// the whole grid.
#include "cc_frontier.h"
#include "cc_static.h"

namespace cc {

__global__ void k_copy16(const int4* __restrict__ src, int4* __restrict__ dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

// First sweep, one lane per vertex: rows of at most kCalibLaneRow entries
// are reduced by their lane (value 1 per entry for MapEdges, vals[w] for
// GatherEdges); longer rows are appended, a wave at a time, to the medium
// list (up to kCalibWaveRow entries) or the heavy list.
constexpr int kCalibLaneRow = 32;
constexpr int kCalibWaveRow = 4096;
constexpr int kCalibBlock = 256;

template <bool GATHER>
__device__ __forceinline__ int32_t edge_value(const int32_t* __restrict__ vals, int32_t w) {
  return GATHER ? vals[w] : (w >= 0 ? 1 : 0);
}

template <bool GATHER, typename I>
__global__ void __launch_bounds__(kCalibBlock) k_edges_reduce(int64_t n, const I* __restrict__ off,
                                                              const int32_t* __restrict__ adj,
                                                              const int32_t* __restrict__ vals,
                                                              int32_t* __restrict__ out, int32_t* heavy,
                                                              int32_t* hcount, int32_t* medium, int32_t* mcount) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    int64_t b = 0, e = 0;
    if (v < n) { b = (int64_t)off[v]; e = (int64_t)off[v + 1]; }
    const int64_t d = e - b;
    wave_append(d > kCalibWaveRow, (int32_t)v, heavy, (uint32_t*)hcount);
    wave_append(d > kCalibLaneRow && d <= kCalibWaveRow, (int32_t)v, medium, (uint32_t*)mcount);
    int32_t acc = 0;
    if (d <= kCalibLaneRow)
      for (int64_t j = b; j < e; ++j) acc += edge_value<GATHER>(vals, adj[j]);
    if (v < n) out[v] = acc;
  }
}

// Medium rows, (kCalibLaneRow, kCalibWaveRow] entries: one wave per row,
// four loads in flight per lane.
template <bool GATHER, typename I>
__global__ void __launch_bounds__(kCalibBlock) k_edges_medium(const int32_t* __restrict__ medium,
                                                              const int32_t* mcount, const I* __restrict__ off,
                                                              const int32_t* __restrict__ adj,
                                                              const int32_t* __restrict__ vals,
                                                              int32_t* __restrict__ out) {
  const int64_t c = *mcount;
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * (kCalibBlock / kWave);
  for (int64_t i = blockIdx.x * (int64_t)(kCalibBlock / kWave) + threadIdx.x / kWave; i < c; i += nwaves) {
    const int32_t u = medium[i];
    const int64_t b = (int64_t)off[u], e = (int64_t)off[u + 1];
    int32_t part = 0;
    for (int64_t j0 = b; j0 < e; j0 += 4 * kWave) {
      int32_t x[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t j = j0 + lane + r * kWave;
        x[r] = j < e ? adj[j] : -1;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (j0 + lane + r * kWave < e) part += edge_value<GATHER>(vals, x[r]);
    }
    part = wave_sum(part);
    if (lane == 0) out[u] = part;
  }
}

// Rows longer than kCalibWaveRow: each wave takes chunks of kCalibChunk
// consecutive entries of the heavy rows' concatenation (hp = degree prefix
// of the heavy list); a lane keeps a running sum while the row of its
// entries stays the same, and whenever some lane reaches a new row the wave
// adds its sums row by row (one atomic per row run), so a row costs one
// atomic per chunk it meets instead of one per 64 entries.
constexpr int64_t kCalibChunk = 4096;

// Adds each lane's `sum` into out[r] for every distinct r >= 0 held by the
// wave's lanes, one atomic per distinct r, and zeroes the sums it added.
__device__ __forceinline__ void wave_add_runs(int32_t r, int32_t& sum, int32_t* out) {
  uint64_t act = __ballot(r >= 0);
  while (act) {
    const int leader = __ffsll((unsigned long long)act) - 1;
    const int32_t lr = __shfl(r, leader, kWave);
    const bool mine = r == lr && r >= 0;
    const int32_t part = wave_sum(mine ? sum : 0);
    if (lane_id() == leader) atomicAdd(out + lr, part);
    act &= ~__ballot(mine);
    if (mine) {
      r = -1;
      sum = 0;
    }
  }
}

template <bool GATHER, typename I>
__global__ void __launch_bounds__(kCalibBlock) k_edges_heavy(const int32_t* __restrict__ heavy, const int32_t* hcount,
                                                             const long long* __restrict__ hp,
                                                             const I* __restrict__ off,
                                                             const int32_t* __restrict__ adj,
                                                             const int32_t* __restrict__ vals,
                                                             int32_t* __restrict__ out) {
  const int64_t c = *hcount;
  if (c == 0) return;
  const long long T = hp[c];
  const int lane = lane_id();
  const int64_t nwaves = (int64_t)gridDim.x * (kCalibBlock / kWave);
  for (int64_t ch = blockIdx.x * (int64_t)(kCalibBlock / kWave) + threadIdx.x / kWave; ch * kCalibChunk < T;
       ch += nwaves) {
    const long long e0 = ch * kCalibChunk;
    const long long e1 = (e0 + kCalibChunk < T) ? e0 + kCalibChunk : T;
    int64_t i = heavy_owner(hp, c, e0);  // the same for every lane
    int32_t cur = -1, sum = 0;
    for (long long e = e0 + lane; __ballot(e < e1); e += kWave) {
      int32_t u = -1, x = 0;
      if (e < e1) {
        while (i + 1 < c && hp[i + 1] <= e) ++i;
        u = heavy[i];
        const int32_t w = adj[(int64_t)off[u] + (e - hp[i])];
        x = GATHER ? vals[w] : (w >= 0 ? 1 : 0);
      }
      const bool moved = cur >= 0 && u != cur;
      if (__ballot(moved)) wave_add_runs(moved ? cur : -1, sum, out);  // zeroes the sums it added
      if (u != cur) {
        cur = u;
        sum = 0;
      }
      sum += x;
    }
    wave_add_runs(cur, sum, out);
  }
}

__global__ void k_zero_two_i32(int32_t* p) { p[0] = p[1] = 0; }

template <bool GATHER, typename I>
static void launch_edges(int64_t n, const I* off, const int32_t* adj, const int32_t* vals, int32_t* out, char* w,
                         size_t hcap, hipStream_t s) {
  int32_t* hcount = (int32_t*)w;
  int32_t* mcount = (int32_t*)w + 1;
  int32_t* heavy = (int32_t*)(w + 256);
  long long* hp = (long long*)(w + 256 + align256(hcap * 4));
  long long* tsum = (long long*)(w + 256 + align256(hcap * 4) + align256((hcap + 1) * 8));
  int32_t* medium = (int32_t*)((char*)tsum + align256((hcap / kHpTile + 3) * 8));
  hipLaunchKernelGGL(k_zero_two_i32, dim3(1), dim3(1), 0, s, hcount);
  hipLaunchKernelGGL((k_edges_reduce<GATHER, I>), dim3(grid_for(n, kCalibBlock, 1 << 16)),
                     dim3(kCalibBlock), 0, s, n, off, adj, vals, out, heavy, hcount, medium, mcount);
  hipLaunchKernelGGL((k_edges_medium<GATHER, I>), dim3(2048), dim3(kCalibBlock), 0, s, (const int32_t*)medium,
                     (const int32_t*)mcount, off, adj, vals, out);
  heavy_prefix<I>(s, heavy, (const int32_t*)hcount, (int64_t)hcap, off, tsum, hp);
  hipLaunchKernelGGL((k_edges_heavy<GATHER, I>), dim3(2048), dim3(kCalibBlock), 0, s, (const int32_t*)heavy,
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
  // heavy list, its degree prefix and tile sums, then the medium list (rows
  // of more than 32 entries: at most m / 32 of them)
  *bytes = 256 + align256(hcap * 4) + align256((hcap + 1) * 8) + align256((hcap / kHpTile + 3) * 8) +
           align256(((size_t)m / 32 + 2) * 4);
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
