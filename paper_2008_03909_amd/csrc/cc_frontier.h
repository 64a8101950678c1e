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

// Atomically set bit x; true iff this call set it.
__device__ __forceinline__ bool bit_claim(uint32_t* bm, int64_t x) {
  const uint32_t b = 1u << (x & 31);
  if (ldu(bm + (x >> 5)) & b) return false;
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

// Sets *flag = 1 once per wave if any active lane saw a change.
__device__ __forceinline__ void wave_flag(bool any, uint32_t* flag) {
  const uint64_t mask = __ballot(any);
  if (mask && lane_id() == __ffsll((unsigned long long)mask) - 1)
    __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Edge visitors over the degree-binned candidate lists written by the
// compaction kernel: op(u, w) for every candidate u and every w in row(u).
template <class Op, typename I>
__global__ void k_visit_thread(const int32_t* __restrict__ cand, const DevScalars* sc, const I* __restrict__ off,
                               const int32_t* __restrict__ adj, Op op, uint32_t* flag) {
  const int64_t cnt = sc->bin_count[0];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool any = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += stride) {
    const int32_t u = cand[i];
    const int64_t e = (int64_t)off[u + 1];
    for (int64_t j = (int64_t)off[u]; j < e; ++j) any |= op(u, adj[j]);
  }
  if (flag) wave_flag(any, flag);
}

template <class Op, typename I>
__global__ void k_visit_wave(const int32_t* __restrict__ big, const DevScalars* sc, const I* __restrict__ off,
                             const int32_t* __restrict__ adj, Op op, uint32_t* flag) {
  const int64_t cnt = sc->bin_count[1];
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int lane = lane_id();
  bool any = false;
  for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < cnt; i += waves) {
    const int32_t u = big[i];
    const int64_t e = (int64_t)off[u + 1];
    for (int64_t j = (int64_t)off[u] + lane; j < e; j += kWave) any |= op(u, adj[j]);
  }
  if (flag) wave_flag(any, flag);
}

template <class Op, typename I>
__global__ void k_visit_block(int64_t n, const int32_t* __restrict__ big, const DevScalars* sc,
                              const I* __restrict__ off, const int32_t* __restrict__ adj, Op op, uint32_t* flag) {
  const int64_t cnt = sc->bin_count[2];
  bool any = false;
  for (int64_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int32_t u = big[n - 1 - i];
    const int64_t e = (int64_t)off[u + 1];
    for (int64_t j = (int64_t)off[u] + threadIdx.x; j < e; j += blockDim.x) any |= op(u, adj[j]);
  }
  if (flag) wave_flag(any, flag);
}

template <class Op, typename I>
inline void visit_candidates(hipStream_t s, int64_t n, const int32_t* cand, const int32_t* big,
                             const DevScalars* sc, const I* off, const int32_t* adj, Op op, uint32_t* flag) {
  hipLaunchKernelGGL((k_visit_thread<Op, I>), dim3(grid_for(n, kFBlock, 4096)), dim3(kFBlock), 0, s, cand, sc, off,
                     adj, op, flag);
  hipLaunchKernelGGL((k_visit_wave<Op, I>), dim3(grid_for(n * kWave, kFBlock, 2048)), dim3(kFBlock), 0, s, big, sc,
                     off, adj, op, flag);
  hipLaunchKernelGGL((k_visit_block<Op, I>), dim3(1024), dim3(kFBlock), 0, s, n, big, sc, off, adj, op, flag);
}

static __global__ void k_set_u32(uint32_t* p, uint32_t v) { *p = v; }

static __global__ void k_fill_u32(uint32_t* p, int64_t count, uint32_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

}  // namespace cc
