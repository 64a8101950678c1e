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
// Short rows are reduced by a wave over 64 rows at a time, long rows in
// edge chunks spread over the grid.
#include "cc_frontier.h"
#include "cc_static.h"

namespace cc {

__global__ void k_copy16(const int4* __restrict__ src, int4* __restrict__ dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

// Rows of up to kCalibWaveRow entries: a wave takes 64 consecutive rows.
// When none of them is longer, their entries are one contiguous run of the
// adjacency; the wave walks it in windows of kCalibWindow entries: every
// lane loads 16 entries of the window (coalesced, all in flight together)
// and stores their values (1 for MapEdges, vals[w] for GatherEdges) in LDS;
// then each lane adds up 16 consecutive values of the window, stepping
// through the row ends it passes and adding each row's part into that
// row's LDS slot.  A wave that holds a longer row (listed for
// k_edges_heavy) walks each of its other rows with the whole wave, or with
// one lane when the row is shorter than a wave.
constexpr int kCalibWaveRow = 4096;
constexpr int kCalibBlock = 256;
constexpr int kCalibPer = 16;
constexpr int kCalibWindow = kCalibPer * 64;

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
  // one padding word after every 16 values, so that the 64 chunks of 16 a
  // lane each reads start in different LDS banks
  __shared__ int32_t win_s[kCalibBlock / kWave][kCalibWindow + kCalibWindow / kCalibPer];
  __shared__ long long end_s[kCalibBlock / kWave][kWave];
  __shared__ int32_t acc_s[kCalibBlock / kWave][kWave];
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  int32_t* win = win_s[wv];
  long long* re = end_s[wv];
  int32_t* acc = acc_s[wv];
  const int64_t nwaves = (int64_t)gridDim.x * (kCalibBlock / kWave);
  for (int64_t wb = blockIdx.x * (int64_t)(kCalibBlock / kWave) + wv; wb * kWave < n; wb += nwaves) {
    const int64_t v = wb * kWave + lane;
    int64_t b = 0, e = 0;
    if (v < n) {
      b = (int64_t)off[v];
      e = (int64_t)off[v + 1];
    }
    const bool heavy_row = (e - b) > kCalibWaveRow;
    wave_append(heavy_row, (int32_t)v, heavy, (uint32_t*)hcount);
    int32_t mine = 0;
    if (__ballot(heavy_row)) {
      // rare: the light rows of this wave are not one run (these waves hold
      // the graph's hubs and many long rows); rows longer than a wave go to
      // k_edges_medium, one wave each, shorter ones are walked by their lane
      const bool wide = !heavy_row && (e - b) > kWave;
      wave_append(wide, (int32_t)v, medium, (uint32_t*)mcount);
      if (!heavy_row && !wide)
        for (int64_t j = b; j < e; ++j) mine += edge_value<GATHER>(vals, adj[j]);
    } else {
      const int last = (int)((n - wb * kWave) < kWave ? (n - wb * kWave) : kWave) - 1;
      const int64_t B = __shfl(b, 0, kWave);
      const int64_t E = __shfl(e, last, kWave);
      re[lane] = lane <= last ? e : E;   // row ends, ascending
      acc[lane] = 0;
      for (int64_t W = B; W < E; W += kCalibWindow) {
        int32_t x[kCalibPer];
#pragma unroll
        for (int r = 0; r < kCalibPer; ++r) {
          const int64_t j = W + lane + (int64_t)r * kWave;
          x[r] = j < E ? adj[j] : 0;
        }
#pragma unroll
        for (int r = 0; r < kCalibPer; ++r) {
          const int64_t j = W + lane + (int64_t)r * kWave;
          const int i = lane + r * kWave;
          win[i + i / kCalibPer] = j < E ? edge_value<GATHER>(vals, x[r]) : 0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int64_t c0 = W + (int64_t)kCalibPer * lane;          // this lane's 16 consecutive entries
        const int64_t c1 = (c0 + kCalibPer < E) ? c0 + kCalibPer : E;
        if (c0 < c1) {
          int lo = 0, hi = kWave - 1;  // first row whose end is past c0
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (re[mid] > c0) hi = mid;
            else lo = mid + 1;
          }
          int row = lo;
          int32_t part = 0;
          for (int64_t j = c0; j < c1; ++j) {
            while (j >= re[row]) {
              if (part) atomicAdd(acc + row, part);
              part = 0;
              ++row;
            }
            const int i = (int)(j - W);
            part += win[i + i / kCalibPer];
          }
          if (part) atomicAdd(acc + row, part);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      mine = acc[lane];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (v < n) out[v] = mine;  // heavy rows start at 0 (k_edges_heavy adds their sums); medium rows are overwritten
  }
}

// Rows of (64, kCalibWaveRow] entries that share a wave with a longer row:
// one wave per row, four loads in flight per lane.
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
  hipLaunchKernelGGL((k_edges_reduce<GATHER, I>), dim3(grid_for(div_up(n, kWave), kCalibBlock / kWave, 1 << 16)),
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
  // of more than 64 entries: at most m / 64 of them)
  *bytes = 256 + align256(hcap * 4) + align256((hcap + 1) * 8) + align256((hcap / kHpTile + 3) * 8) +
           align256(((size_t)m / kWave + 2) * 4);
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
