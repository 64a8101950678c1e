// Frontier helpers shared by the BFS and LDD samplers and the round-based
// finishes: bitmaps, wave-aggregated queue appends, edge visitors over the
// degree-binned candidate lists.
#pragma once
#include "cc_device.h"
#include "cc_internal.h"

namespace cc {

constexpr int kFBlock = 256;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Plain read of a bitmap bit (used where a stale 0 only costs an atomic).
__device__ __forceinline__ bool bit_get(const uint32_t* bm, int64_t x) { return (bm[x >> 5] >> (x & 31)) & 1u; }

// Atomically set bit x; true iff this call set it.  Bits only ever go from
// 0 to 1, so a plain (possibly stale) read that already shows the bit is
// conclusive and saves the atomic; a stale 0 falls through to it.
__device__ __forceinline__ bool bit_claim(uint32_t* bm, int64_t x) {
  const uint32_t b = 1u << (x & 31);
  if (bm[x >> 5] & b) return false;
  return !(aor(bm + (x >> 5), b) & b);
}

// Appends `val` for every active lane with take=true; one atomic per wave.
__device__ __forceinline__ void wave_append(bool take, int32_t val, int32_t* q, uint32_t* cnt) {
  const uint64_t mask = __ballot(take);
  if (!mask) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  uint32_t base = 0;
  if (lane_id() == leader)
    base = __hip_atomic_fetch_add(cnt, (uint32_t)__popcll(mask), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, leader, kWave);
  if (take) q[base + (uint32_t)__popcll(mask & lanemask_lt())] = val;
}

__device__ __forceinline__ void wave_append_pair(bool take, int32_t a, int32_t b, int32_t* qa, int32_t* qb,
                                                 unsigned long long* cnt) {
  const uint64_t mask = __ballot(take);
  if (!mask) return;
  const int leader = __ffsll((unsigned long long)mask) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader)
    base = __hip_atomic_fetch_add(cnt, (unsigned long long)__popcll(mask), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, leader, kWave);
  if (take) {
    const unsigned long long p = base + (unsigned long long)__popcll(mask & lanemask_lt());
    qa[p] = a;
    qb[p] = b;
  }
}

// Wave-private output buffer in LDS: appends cost LDS writes; the global
// queue counter is bumped once per flush (at most kWaveQCap entries).  Every
// call must be made by all 64 lanes of the wave together (uniform control
// flow), since `cnt` is a wave-uniform register.
constexpr int kWaveQCap = 512;

struct WaveQ {
  int32_t* buf;  // this wave's kWaveQCap-entry LDS slice
  int cnt;
};

__device__ __forceinline__ void wq_flush(WaveQ& q, int32_t* gq, uint32_t* gcnt) {
  if (q.cnt == 0) return;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t base = 0;
  if (lane_id() == 0)
    base = __hip_atomic_fetch_add(gcnt, (uint32_t)q.cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  base = __shfl(base, 0, kWave);
  for (int i = lane_id(); i < q.cnt; i += kWave) gq[base + i] = q.buf[i];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  q.cnt = 0;
}

__device__ __forceinline__ void wq_push(WaveQ& q, bool take, int32_t val, int32_t* gq, uint32_t* gcnt) {
  const uint64_t m = __ballot(take);
  if (take) q.buf[q.cnt + __popcll(m & lanemask_lt())] = val;
  q.cnt += __popcll(m);
  if (q.cnt > kWaveQCap - kWave) wq_flush(q, gq, gcnt);
}

// Sets *flag = 1 once per wave if any active lane saw a change.
__device__ __forceinline__ void wave_flag(bool any, uint32_t* flag) {
  const uint64_t mask = __ballot(any);
  if (mask && lane_id() == __ffsll((unsigned long long)mask) - 1)
    __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Degree bins of the candidate lists and of frontier vertices.
constexpr int kThrWave = 32;      // degree <= 32: one thread per vertex
constexpr int kThrBlock = 256;    // <= 256: one wave; <= kThrGrid: one block
constexpr int kThrGrid = 4096;    // larger: the whole grid, edge-balanced
constexpr int kHeavyFrontier = 256;  // frontier rows above this go to the grid kernel

// Capacity of a heavy list: vertices whose degree exceeds kHeavyFrontier.
inline size_t heavy_cap(int64_t m) { return (size_t)(m / kHeavyFrontier) + 2; }

// Exclusive prefix of the degrees of a vertex list whose length lives on the
// device: hp[i] = sum of deg(list[j]) for j < i, hp[count] = total.  Three
// launches: per-tile sums, one-block scan of the tile sums, tile scans.  The
// grid is sized for the list's capacity; surplus blocks exit at once.
constexpr int kHpTile = 1024;

__device__ __forceinline__ long long block_excl_scan_ll(long long x, long long* total) {
  __shared__ long long wsum[1024 / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  long long inc = x;
  for (int o = 1; o < kWave; o <<= 1) {
    const long long y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  long long before = 0, all = 0;
  for (int q = 0; q < nw; ++q) {
    if (q < w) before += wsum[q];
    all += wsum[q];
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

template <typename I>
__device__ __forceinline__ long long list_deg(const int32_t* list, int64_t i, int64_t c, const I* off) {
  if (i >= c) return 0;
  const int32_t u = list[i];
  return (long long)off[u + 1] - (long long)off[u];
}

template <typename I>
__global__ void __launch_bounds__(kHpTile) k_hp_tiles(const int32_t* __restrict__ list, const int32_t* count_ptr,
                                                      const I* __restrict__ off, long long* __restrict__ tsum) {
  const int64_t c = *count_ptr;
  const int64_t i = blockIdx.x * (int64_t)kHpTile + threadIdx.x;
  if ((int64_t)blockIdx.x * kHpTile >= c) return;
  long long total;
  block_excl_scan_ll(list_deg(list, i, c, off), &total);
  if (threadIdx.x == 0) tsum[blockIdx.x] = total;
}

[[maybe_unused]] static __global__ void __launch_bounds__(kHpTile) k_hp_top(const int32_t* count_ptr, long long* tsum) {
  const int64_t c = *count_ptr;
  const int64_t tiles = (c + kHpTile - 1) / kHpTile;
  long long carry = 0;
  for (int64_t base = 0; base < tiles; base += kHpTile) {
    const int64_t i = base + threadIdx.x;
    const long long x = i < tiles ? tsum[i] : 0;
    long long total;
    const long long ex = block_excl_scan_ll(x, &total);
    if (i < tiles) tsum[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) tsum[tiles] = carry;  // grand total after the tile offsets
}

template <typename I>
__global__ void __launch_bounds__(kHpTile) k_hp_down(const int32_t* __restrict__ list, const int32_t* count_ptr,
                                                     const I* __restrict__ off, const long long* __restrict__ tsum,
                                                     long long* __restrict__ hp) {
  const int64_t c = *count_ptr;
  if ((int64_t)blockIdx.x * kHpTile >= c) {
    if (blockIdx.x == 0 && threadIdx.x == 0) hp[0] = 0;
    return;
  }
  const int64_t i = blockIdx.x * (int64_t)kHpTile + threadIdx.x;
  long long total;
  const long long ex = block_excl_scan_ll(list_deg(list, i, c, off), &total);
  if (i < c) hp[i] = tsum[blockIdx.x] + ex;
  if (i == c - 1) hp[c] = tsum[(c + kHpTile - 1) / kHpTile];
}

// Launches the three prefix kernels for a list of capacity `cap` (tsum holds
// cap / kHpTile + 2 entries).
template <typename I>
inline void heavy_prefix(hipStream_t s, const int32_t* list, const int32_t* count_ptr, int64_t cap, const I* off,
                         long long* tsum, long long* hp) {
  const unsigned tiles = (unsigned)((cap + kHpTile - 1) / kHpTile);
  hipLaunchKernelGGL(k_hp_tiles<I>, dim3(tiles ? tiles : 1), dim3(kHpTile), 0, s, list, count_ptr, off, tsum);
  hipLaunchKernelGGL(k_hp_top, dim3(1), dim3(kHpTile), 0, s, count_ptr, tsum);
  hipLaunchKernelGGL(k_hp_down<I>, dim3(tiles ? tiles : 1), dim3(kHpTile), 0, s, list, count_ptr, off,
                     (const long long*)tsum, hp);
}

// Largest i in [0, c) with hp[i] <= e (hp ascending, hp[0] = 0 <= e).
__device__ __forceinline__ int64_t heavy_owner(const long long* hp, int64_t c, long long e) {
  int64_t lo = 0, hi = c - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (hp[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Owner of edge e for a wave that covers the tile [e0, e0 + 64): one binary
// search for the tile start (the same for every lane), then each lane steps
// forward; heavy rows are longer than a tile, so that is at most one step.
__device__ __forceinline__ int64_t heavy_owner_tile(const long long* hp, int64_t c, long long e0, long long e) {
  int64_t i = heavy_owner(hp, c, e0);
  while (i + 1 < c && hp[i + 1] <= e) ++i;
  return i;
}

// Edge visitors over the degree-binned candidate lists written by the
// compaction: op(u, w, j) for every candidate u and every entry j of row(u),
// w = adj[j].  Thread bin: cand front; wave bin: big front; block bin: big
// back; grid bin: the heavy list, whose edges are spread evenly over all of
// the bin's blocks.  Each part runs as block `bid` of `nb` blocks, so the
// four can share one launch (k_visit_all) or run as kernels of their own.
template <class Op, typename I>
__device__ __forceinline__ void visit_thread_part(int64_t bid, int64_t nb, const int32_t* __restrict__ cand,
                                                  const int32_t* bins, const I* __restrict__ off,
                                                  const int32_t* __restrict__ adj, const Op& op, uint32_t* flag) {
  const int64_t cnt = bins[0];
  const int64_t stride = nb * blockDim.x;
  bool any = false;
  for (int64_t i = bid * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += stride) {
    const int32_t u = cand[i];
    const int64_t e = (int64_t)off[u + 1];
    for (int64_t j = (int64_t)off[u]; j < e; ++j) any |= op(u, adj[j], j);
  }
  if (flag) wave_flag(any, flag);
}

template <class Op, typename I>
__device__ __forceinline__ void visit_wave_part(int64_t bid, int64_t nb, const int32_t* __restrict__ big,
                                                const int32_t* bins, const I* __restrict__ off,
                                                const int32_t* __restrict__ adj, const Op& op, uint32_t* flag) {
  const int64_t cnt = bins[1];
  const int64_t waves = nb * (blockDim.x / kWave);
  const int lane = lane_id();
  bool any = false;
  for (int64_t i = bid * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < cnt; i += waves) {
    const int32_t u = big[i];
    const int64_t e = (int64_t)off[u + 1];
    for (int64_t j = (int64_t)off[u] + lane; j < e; j += kWave) any |= op(u, adj[j], j);
  }
  if (flag) wave_flag(any, flag);
}

template <class Op, typename I>
__device__ __forceinline__ void visit_block_part(int64_t bid, int64_t nb, int64_t n, const int32_t* __restrict__ big,
                                                 const int32_t* bins, const I* __restrict__ off,
                                                 const int32_t* __restrict__ adj, const Op& op, uint32_t* flag) {
  const int64_t cnt = bins[2];
  bool any = false;
  for (int64_t i = bid; i < cnt; i += nb) {
    const int32_t u = big[n - 1 - i];
    const int64_t e = (int64_t)off[u + 1];
    for (int64_t j = (int64_t)off[u] + threadIdx.x; j < e; j += blockDim.x) any |= op(u, adj[j], j);
  }
  if (flag) wave_flag(any, flag);
}

template <class Op, typename I>
__device__ __forceinline__ void visit_heavy_part(int64_t bid, int64_t nb, const int32_t* __restrict__ hlist,
                                                 const int32_t* count_ptr, const long long* __restrict__ hp,
                                                 const I* __restrict__ off, const int32_t* __restrict__ adj,
                                                 const Op& op, uint32_t* flag) {
  const int64_t c = *count_ptr;
  bool any = false;
  if (c > 0) {
    const long long T = hp[c];  // the list's edge total
    const int64_t stride = nb * blockDim.x;
    for (long long base = bid * (int64_t)blockDim.x; base < T; base += stride) {
      const long long e0 = base + (threadIdx.x / kWave) * kWave;
      const long long e = base + threadIdx.x;
      if (e0 >= T) continue;
      if (e < T) {
        const int64_t i = heavy_owner_tile(hp, c, e0, e);
        const int32_t u = hlist[i];
        const int64_t j = (int64_t)off[u] + (e - hp[i]);
        any |= op(u, adj[j], j);
      }
    }
  }
  if (flag) wave_flag(any, flag);
}

template <class Op, typename I>
__global__ void k_visit_thread(const int32_t* __restrict__ cand, const int32_t* bins, const I* __restrict__ off,
                               const int32_t* __restrict__ adj, Op op, uint32_t* flag) {
  visit_thread_part<Op, I>(blockIdx.x, gridDim.x, cand, bins, off, adj, op, flag);
}

template <class Op, typename I>
__global__ void k_visit_wave(const int32_t* __restrict__ big, const int32_t* bins, const I* __restrict__ off,
                             const int32_t* __restrict__ adj, Op op, uint32_t* flag) {
  visit_wave_part<Op, I>(blockIdx.x, gridDim.x, big, bins, off, adj, op, flag);
}

template <class Op, typename I>
__global__ void k_visit_block(int64_t n, const int32_t* __restrict__ big, const int32_t* bins,
                              const I* __restrict__ off, const int32_t* __restrict__ adj, Op op, uint32_t* flag) {
  visit_block_part<Op, I>(blockIdx.x, gridDim.x, n, big, bins, off, adj, op, flag);
}

template <class Op, typename I>
__global__ void k_visit_heavy(const int32_t* __restrict__ hlist, const int32_t* count_ptr,
                              const long long* __restrict__ hp, const I* __restrict__ off,
                              const int32_t* __restrict__ adj, Op op, uint32_t* flag) {
  visit_heavy_part<Op, I>(blockIdx.x, gridDim.x, hlist, count_ptr, hp, off, adj, op, flag);
}

// All four bins in one launch: blocks [0, g0) take the thread bin, the next
// g1 the wave bin, the next g2 the block bin, the rest the grid bin.
template <class Op, typename I>
__global__ void k_visit_all(int64_t n, int64_t g0, int64_t g1, int64_t g2, const int32_t* __restrict__ cand,
                            const int32_t* __restrict__ big, const int32_t* __restrict__ heavy,
                            const long long* __restrict__ hp, const int32_t* bins, const I* __restrict__ off,
                            const int32_t* __restrict__ adj, Op op, uint32_t* flag) {
  int64_t b = blockIdx.x;
  if (b < g0) return visit_thread_part<Op, I>(b, g0, cand, bins, off, adj, op, flag);
  b -= g0;
  if (b < g1) return visit_wave_part<Op, I>(b, g1, big, bins, off, adj, op, flag);
  b -= g1;
  if (b < g2) return visit_block_part<Op, I>(b, g2, n, big, bins, off, adj, op, flag);
  b -= g2;
  visit_heavy_part<Op, I>(b, (int64_t)gridDim.x - g0 - g1 - g2, heavy, &bins[3], hp, off, adj, op, flag);
}

// Degree-binned vertex lists: the candidates of one static call, or a
// frontier in the same layout.
struct CandLists {
  int64_t n;
  const int32_t* cand;    // thread bin
  const int32_t* big;     // wave bin (front), block bin (back)
  const int32_t* heavy;   // grid bin
  const long long* hp;    // degree prefix of the grid bin
  const int32_t* bins;    // the four bins' lengths (device)
};

// Blocks of each bin's part in a combined launch over lists of n vertices:
// grid-stride parts, enough blocks to fill the device, few enough that an
// almost empty list (k-out leaves a few thousand candidates) costs little.
inline void visit_grids(int64_t n, int64_t g[4]) {
  g[0] = grid_for(n, kFBlock, 2048);
  g[1] = grid_for(n * kWave, kFBlock, 1024);
  g[2] = 512;
  g[3] = 1024;
}

template <class Op, typename I>
inline void visit_candidates(hipStream_t s, const CandLists& L, const I* off, const int32_t* adj, Op op,
                             uint32_t* flag) {
  int64_t g[4];
  visit_grids(L.n, g);
  hipLaunchKernelGGL((k_visit_all<Op, I>), dim3((unsigned)(g[0] + g[1] + g[2] + g[3])), dim3(kFBlock), 0, s, L.n,
                     g[0], g[1], g[2], L.cand, L.big, L.heavy, L.hp, L.bins, off, adj, op, flag);
}

[[maybe_unused]] static __global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

[[maybe_unused]] static __global__ void k_fill_u32(uint32_t* p, int64_t count, uint32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

}  // namespace cc
