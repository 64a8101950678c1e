// Sampling by breadth-first search and by low-diameter decomposition
// (ConnectIt Section 3.2; appendix "Sampling Schemes").
//
// BFS sampling: up to `bfs_tries` sources s_t = splitmix64(key_bfs, t) mod n;
// a direction-optimizing BFS (Beamer et al.) marks the component of s_t in a
// visited bitmap; the try succeeds iff more than n/10 vertices were reached
// (10 * reached > n).  On success the reached vertices are labelled with
// their minimum member (a star rooted at the component minimum, so every
// later link still points to a smaller id); otherwise the labelling stays
// the identity.
//
// LDD sampling: one round of Miller-Peng-Xu.  Each vertex draws
// delta_v = -ln(U_v)/beta; start_v = floor(delta_max - delta_v).  With the
// paper's default ordering (no permutation) the sorted start times are handed
// out in vertex-id order: vertex ids [S_{r-1}, S_r) wake at round r, where
// S_r counts vertices with start <= r.  Round r: unvisited wakers become
// centres, then every frontier vertex claims its unvisited neighbours for
// its cluster (first claim wins).  Clusters are then relabelled to their
// minimum member.
#include <cmath>
#include <vector>

#include "cc_frontier.h"
#include "cc_static.h"

namespace cc {

cc_status pull_scalars(StaticArgs& a) {
  CC_HIP(hipMemcpyAsync(a.ctx->host, a.ctx->dev, sizeof(DevScalars), hipMemcpyDeviceToHost, a.s));
  CC_HIP(hipStreamSynchronize(a.s));
  return CC_OK;
}

// ---- BFS --------------------------------------------------------------------
//
// The levels run without host synchronisation: a level is a prologue kernel
// (one block decides the direction from device counters and resets them;
// every block clears the next frontier bitmap), one expansion kernel that
// runs the top-down or the bottom-up step as the prologue decided (or
// nothing once the search is finished), and, for graphs with vertices above
// kHeavyFrontier, the degree prefix and grid expansion of heavy frontier
// rows.  The host enqueues levels in growing batches and, after each batch,
// a 16-byte snapshot copy into pinned memory; it waits on the previous
// batch's snapshot while the current batch runs, and stops once a snapshot
// says the search finished (the levels queued after it do nothing).

enum : uint32_t { kBfsTopDown = 0, kBfsBottomUp = 1, kBfsDone = 2, kBfsSmall = 3 };
constexpr int kSmallEdges = 4096;      // single-block levels while a frontier scans at most this many entries
constexpr int kSmallLevels = 2048;     // at most this many single-block levels per launch
constexpr int kBfsParts = 2048;        // per-block degree sums of the next frontier
constexpr int kBfsStepBlocks = 1024;   // fpart[0, 1024): step; [1024, 2048): heavy rows
constexpr double kBeamerAlpha = 15.0, kBeamerBeta = 18.0;   // direction-switch constants (Beamer et al.)

template <typename I>
__global__ void k_bfs_start(int32_t s, const I* off, uint32_t* vis, uint32_t* fc, int32_t* q0, DevScalars* sc) {
  vis[s >> 5] |= 1u << (s & 31);
  fc[s >> 5] |= 1u << (s & 31);
  q0[0] = s;
  const long long d = (long long)off[s + 1] - (long long)off[s];
  sc->qcount[0] = 1;
  sc->qcount[1] = 0;
  sc->frontier_edges = d;
  sc->seen_edges = d;
  sc->bfs_mode = kBfsTopDown;
  sc->bfs_level = 0;
  sc->reached = 1;
  sc->heavy_pack = 0ull;
}

// Heavy frontier rows are listed with their edge offsets reserved at the
// same time: one 64-bit atomic per wave adds (rows << 36 | edges) to `pack`,
// so slot i gets hp[i] = the edges listed before it and the offsets come out
// sorted by slot -- the prefix the grid kernel searches, with no separate
// scan.  A level lists at most m / 256 + 2 rows holding at most m entries,
// so both fields fit while m < 2^36 (BFS and LDD refuse larger graphs).
constexpr int kPackShift = 36;
constexpr unsigned long long kPackEdges = (1ull << kPackShift) - 1;

// Lists lane's row u (degree d) if heavy_row; called by the whole wave.
__device__ __forceinline__ void heavy_reserve(bool heavy_row, int32_t u, int64_t d, int32_t* heavy, long long* hp,
                                              unsigned long long* pack) {
  const uint64_t mh = __ballot(heavy_row);
  if (!mh) return;  // rare: one atomic per wave with a heavy row
  const int lane = lane_id();
  long long hd = heavy_row ? d : 0;
  for (int o = 1; o < kWave; o <<= 1) {
    const long long y = __shfl_up(hd, o, kWave);
    if (lane >= o) hd += y;
  }
  const long long hsum = __shfl(hd, kWave - 1, kWave);
  const int leader = __ffsll((unsigned long long)mh) - 1;
  unsigned long long old = 0;
  if (lane == leader)
    old = __hip_atomic_fetch_add(pack, ((unsigned long long)__popcll(mh) << kPackShift) | (unsigned long long)hsum,
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  old = __shfl(old, leader, kWave);
  if (heavy_row) {
    const long long slot = (long long)(old >> kPackShift) + __popcll(mh & lanemask_lt());
    heavy[slot] = u;
    hp[slot] = (long long)(old & kPackEdges) + hd - d;
  }
}

__device__ __forceinline__ long long block_sum_ll(long long x, long long* red) {
  x = wave_sum(x);
  if (lane_id() == 0) red[threadIdx.x / kWave] = x;
  __syncthreads();
  long long s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += red[w];
  return s;
}

// Level prologue.  Block 0: degree sum of the frontier just produced (from
// the per-block partials of the previous level), reached += its size,
// direction for the coming level, counters of the next frontier reset.
// Every block: clears the next frontier bitmap.
__global__ void __launch_bounds__(kFBlock) k_bfs_begin(int64_t words, uint32_t* fn, DevScalars* sc, int cur,
                                                       const long long* __restrict__ fpart, int64_t n, int64_t m,
                                                       int level_cap) {
  __shared__ long long red[kFBlock / kWave];
  if (blockIdx.x == 0) {
    long long s = 0;
    for (int i = threadIdx.x; i < kBfsParts; i += kFBlock) s += fpart[i];
    s = block_sum_ll(s, red);
    if (threadIdx.x == 0 && sc->bfs_mode != kBfsDone) {
      const int64_t nf = sc->qcount[cur];
      long long mf = sc->frontier_edges;
      if (sc->bfs_level > 0) {   // the frontier was produced by the previous level
        mf = s;
        sc->reached += nf;
        sc->seen_edges += mf;
        sc->frontier_edges = mf;
      }
      uint32_t mode = sc->bfs_mode;
      if (nf == 0 || (level_cap > 0 && sc->bfs_level >= level_cap)) {
        mode = kBfsDone;
      } else if (mode == kBfsTopDown && (double)mf > (double)(m - sc->seen_edges + mf) / kBeamerAlpha) {
        mode = kBfsBottomUp;
      } else if (mode == kBfsBottomUp && (double)nf < (double)n / kBeamerBeta) {
        mode = kBfsTopDown;
      } else if (mode == kBfsSmall) {
        mode = kBfsTopDown;
      }
      // a frontier this small is expanded level after level by one block
      if (mode == kBfsTopDown && mf <= kSmallEdges && (level_cap <= 0)) mode = kBfsSmall;
      sc->bfs_mode = mode;
      sc->qcount[cur ^ 1] = 0;
      sc->heavy_pack = 0ull;
      if (mode != kBfsDone) sc->bfs_level += 1;
    }
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += stride) fn[i] = 0u;
}

// Small frontiers (degree sum <= kSmallEdges): one block expands level after
// level, with the frontier's degree prefix in LDS and __syncthreads between
// levels, while the frontier stays that small (at most kSmallLevels levels).
// Queues alternate between qin and qout; the last frontier produced (not yet
// expanded) is left in qout with its bits in fn, as if one level had run,
// and the levels, reached vertices and scanned edges of the internal levels
// are added to the device counters.  Returns that frontier's degree sum.
template <typename I>
__device__ long long bfs_small_levels(const I* __restrict__ off, const int32_t* __restrict__ adj, uint32_t* vis,
                                      uint32_t* fn, const int32_t* qin0, uint32_t f0, int32_t* qout0,
                                      uint32_t* cnt_out, DevScalars* sc, int2* tree) {
  __shared__ int32_t spre[kSmallEdges + 2];
  __shared__ long long stsum[kFBlock];
  __shared__ long long stotal;
  __shared__ int32_t snn;
  const int t = threadIdx.x;
  int32_t* qa = const_cast<int32_t*>(qin0);
  int32_t* qb = qout0;
  int64_t f = f0;
  int levels = 0;
  long long reached_add = 0, seen_add = 0, fe = 0;
  while (true) {
    // degree sum of the current frontier (contiguous chunk per thread)
    const int64_t chunk = (f + kFBlock - 1) / kFBlock;
    const int64_t i0 = t * chunk < f ? t * chunk : f;
    const int64_t i1 = i0 + chunk < f ? i0 + chunk : f;
    long long sum = 0;
    for (int64_t i = i0; i < i1; ++i) sum += (long long)off[qa[i] + 1] - (long long)off[qa[i]];
    stsum[t] = sum;
    __syncthreads();
    if (t == 0) {
      long long acc = 0;
      for (int i = 0; i < kFBlock; ++i) {
        const long long x = stsum[i];
        stsum[i] = acc;
        acc += x;
      }
      stotal = acc;
      snn = 0;
    }
    __syncthreads();
    fe = stotal;
    if (f == 0 || (levels > 0 && (fe > kSmallEdges || levels >= kSmallLevels))) break;
    if (levels > 0) {            // an internally produced frontier about to be expanded
      reached_add += f;
      seen_add += fe;
    }
    {
      int32_t acc = (int32_t)stsum[t];
      for (int64_t i = i0; i < i1; ++i) {
        spre[i] = acc;
        acc += (int32_t)((long long)off[qa[i] + 1] - (long long)off[qa[i]]);
      }
      if (t == 0) spre[f] = (int32_t)fe;
    }
    __syncthreads();
    for (int32_t e = t; e < (int32_t)fe; e += kFBlock) {
      int64_t lo = 0, hi = f - 1;   // owner: largest i with spre[i] <= e
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (spre[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      const int32_t x = qa[lo];
      const int32_t w = adj[(int64_t)off[x] + (e - spre[lo])];
      if (bit_claim(vis, w)) {
        qb[atomicAdd(&snn, 1)] = w;
        if (tree) tree[w] = make_int2(x, w);
      }
    }
    __syncthreads();
    f = snn;
    ++levels;
    int32_t* tq = qa;
    qa = qb;
    qb = tq;
    __syncthreads();
  }
  // the current frontier (qa, f entries) is the output
  if (qa != qout0)
    for (int64_t i = t; i < f; i += kFBlock) qout0[i] = qa[i];
  for (int64_t i = t; i < f; i += kFBlock) {
    const int32_t w = qa[i];
    aor(fn + (w >> 5), 1u << (w & 31));
  }
  if (t == 0) {
    *cnt_out = (uint32_t)f;
    sc->bfs_level += levels - 1;
    sc->reached += reached_add;
    sc->seen_edges += seen_add;
  }
  return t == 0 ? fe : 0;
}

// One BFS level.  Top-down: the wave-balanced expansion of the frontier
// queue (rows above kHeavyFrontier deferred); claimed vertices are appended
// to the next queue and marked in the next bitmap.  Bottom-up: each
// unvisited vertex looks for a neighbour in the current bitmap; lanes map to
// consecutive vertices, so the 32 bits of a bitmap word belong to one wave,
// which writes the word itself (no atomics).  Both write the degree sum of
// the vertices they add to fpart[blockIdx].
template <typename I>
__global__ void __launch_bounds__(kFBlock) k_bfs_step(int64_t n, const I* __restrict__ off,
                                                      const int32_t* __restrict__ adj, uint32_t* vis,
                                                      const uint32_t* __restrict__ fc, uint32_t* fn,
                                                      const int32_t* __restrict__ qin, const uint32_t* cnt_in,
                                                      int32_t* qout, uint32_t* cnt_out, int32_t* heavy,
                                                      long long* hp, DevScalars* sc,
                                                      long long* __restrict__ fpart, int2* tree) {
  constexpr int W = kFBlock / kWave;
  __shared__ int32_t qbuf[W][kWaveQCap];
  __shared__ int32_t tpre[W][kWave + 1];
  __shared__ int64_t tbeg[W][kWave];
  __shared__ int32_t tu[W][kWave];
  __shared__ long long red[W];
  const uint32_t mode = sc->bfs_mode;
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  WaveQ q{qbuf[wv], 0};
  long long added = 0;
  if (mode == kBfsSmall) {
    if (blockIdx.x == 0) added = bfs_small_levels<I>(off, adj, vis, fn, qin, *cnt_in, qout, cnt_out, sc, tree);
  } else if (mode == kBfsTopDown) {
    const int64_t cnt = *cnt_in;
    const int64_t tiles = (cnt + kWave - 1) / kWave;
    const int64_t waves = (int64_t)gridDim.x * W;
    for (int64_t tile = blockIdx.x * (int64_t)W + wv; tile < tiles; tile += waves) {
      const int64_t idx = tile * kWave + lane;
      int32_t u = 0;
      int64_t b = 0, d = 0;
      if (idx < cnt) {
        u = qin[idx];
        b = (int64_t)off[u];
        d = (int64_t)off[u + 1] - b;
      }
      const bool heavy_row = d > kHeavyFrontier;
      heavy_reserve(heavy_row, u, d, heavy, hp, &sc->heavy_pack);
      if (heavy_row) d = 0;
      int32_t inc = (int32_t)d;
      for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += y;
      }
      const int32_t total = __shfl(inc, kWave - 1, kWave);
      tpre[wv][lane] = inc - (int32_t)d;
      if (lane == kWave - 1) tpre[wv][kWave] = total;
      tbeg[wv][lane] = b;
      tu[wv][lane] = u;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int32_t e0 = 0; e0 < total; e0 += kWave) {
        const int32_t e = e0 + lane;
        bool got = false;
        int32_t w = 0;
        if (e < total) {
          int lo = 0, hi = kWave - 1;  // last row whose start <= e
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tpre[wv][mid] <= e) lo = mid;
            else hi = mid - 1;
          }
          w = adj[tbeg[wv][lo] + (e - tpre[wv][lo])];
          got = bit_claim(vis, w);
          if (got) {
            aor(fn + (w >> 5), 1u << (w & 31));
            added += (long long)off[w + 1] - (long long)off[w];
            if (tree) tree[w] = make_int2(tu[wv][lo], w);
          }
        }
        wq_push(q, got, w, qout, cnt_out);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  } else if (mode == kBfsBottomUp) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ++sc->bu_rounds;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
      const int64_t v = base + threadIdx.x;
      bool found = false;
      if (v < n && !bit_get(vis, v)) {
        const int64_t e = (int64_t)off[v + 1];
        const int64_t b = (int64_t)off[v];
        for (int64_t j = b; j < e; ++j) {
          const int32_t x = adj[j];
          if (bit_get(fc, x)) {
            found = true;
            if (tree) tree[v] = make_int2(x, (int32_t)v);
            break;
          }
        }
        if (found) added += e - b;
      }
      // base is a multiple of 256, so lanes 0-31 and 32-63 each cover one
      // whole bitmap word; its owner lane writes it
      const uint64_t bits = __ballot(found);
      if ((lane & 31) == 0 && v < n) {
        const uint32_t wbits = (uint32_t)(bits >> (lane & 32));
        if (wbits) {
          vis[v >> 5] |= wbits;
          fn[v >> 5] = wbits;
        }
      }
      wq_push(q, found, (int32_t)v, qout, cnt_out);
    }
  }
  wq_flush(q, qout, cnt_out);
  added = wave_sum(added);
  if (lane == 0) red[wv] = added;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int w = 0; w < W; ++w) s += red[w];
    fpart[blockIdx.x] = s;
  }
}

// Heavy frontier rows (top-down levels only), spread evenly over the grid;
// degree sums of the added vertices to fpart[kBfsStepBlocks + blockIdx].
template <typename I>
__global__ void __launch_bounds__(kFBlock) k_bfs_heavy(const int32_t* __restrict__ heavy,
                                                       const long long* __restrict__ hp, const I* __restrict__ off,
                                                       const int32_t* __restrict__ adj, uint32_t* vis, uint32_t* fn,
                                                       int32_t* qout, uint32_t* cnt_out, const DevScalars* sc,
                                                       long long* __restrict__ fpart, int2* tree) {
  __shared__ int32_t qbuf[kFBlock / kWave][kWaveQCap];
  __shared__ long long red[kFBlock / kWave];
  WaveQ q{qbuf[threadIdx.x / kWave], 0};
  const unsigned long long pk = sc->bfs_mode == kBfsTopDown ? sc->heavy_pack : 0ull;
  const int64_t c = (int64_t)(pk >> kPackShift);
  long long added = 0;
  if (c > 0) {
    const long long T = (long long)(pk & kPackEdges);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (long long base = blockIdx.x * (int64_t)blockDim.x; base < T; base += stride) {
      const long long e = base + threadIdx.x;
      const long long e0 = base + (threadIdx.x / kWave) * kWave;
      bool got = false;
      int32_t w = 0;
      if (e < T) {
        const int64_t i = heavy_owner_tile(hp, c, e0, e);
        const int32_t u = heavy[i];
        w = adj[(int64_t)off[u] + (e - hp[i])];
        got = bit_claim(vis, w);
        if (got) {
          aor(fn + (w >> 5), 1u << (w & 31));
          added += (long long)off[w + 1] - (long long)off[w];
          if (tree) tree[w] = make_int2(u, w);
        }
      }
      wq_push(q, got, w, qout, cnt_out);
    }
    wq_flush(q, qout, cnt_out);
  }
  added = wave_sum(added);
  if (lane_id() == 0) red[threadIdx.x / kWave] = added;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int w = 0; w < kFBlock / kWave; ++w) s += red[w];
    fpart[kBfsStepBlocks + blockIdx.x] = s;
  }
}

template <typename I>
__global__ void __launch_bounds__(kFBlock) k_count_heavy(int64_t n, const I* __restrict__ off,
                                                         unsigned long long* out) {
  __shared__ long long red[kFBlock / kWave];
  long long c = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride)
    c += ((int64_t)off[v + 1] - (int64_t)off[v]) > kHeavyFrontier;
  c = block_sum_ll(c, red);
  if (threadIdx.x == 0 && c) atomicAdd(out, (unsigned long long)c);
}

__global__ void k_zero_u64_one(unsigned long long* p) { *p = 0ull; }

template <typename I>
cc_status count_heavy(StaticArgs& a) {
  if (a.heavy_vertices >= 0) return CC_OK;
  unsigned long long* d = &a.ctx->dev->heavy_count;
  hipLaunchKernelGGL(k_zero_u64_one, dim3(1), dim3(1), 0, a.s, d);
  hipLaunchKernelGGL(k_count_heavy<I>, dim3(grid_for(a.n, kFBlock, 1024)), dim3(kFBlock), 0, a.s, a.n,
                     (const I*)a.off, d);
  CC_LAUNCH_CHECK();
  unsigned long long h = 0;
  CC_HIP(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, a.s));
  CC_HIP(hipStreamSynchronize(a.s));
  a.heavy_vertices = (int64_t)h;
  return CC_OK;
}

// Frontier expansion (BFS top-down step, LDD cluster growth), load-balanced
// within each wave: a wave takes 64 frontier vertices, concatenates their
// rows (exclusive scan of the degrees across lanes) and walks the joint edge
// list 64 edges at a time; each lane finds the row of its edge by a binary
// search over the 64 row starts in LDS.  Rows above kHeavyFrontier are
// deferred to the grid kernel.  Claimed vertices go through a wave-private
// LDS buffer, so the output queue's counter is bumped once per flush.

// LDD round direction, after the direction-optimizing rule of BFS: bottom-up
// when the frontier's edges exceed 1/kLddAlpha of the edges not yet
// expanded and n/kLddGamma (a bottom-up round visits every vertex, so a
// frontier with fewer edges than that is cheaper top-down).  Every kernel
// of a round evaluates it from the same scalars (final once the round's
// wake has run), so they all agree without a host round trip.
constexpr long long kLddAlpha = 14, kLddGamma = 4;

__device__ __forceinline__ bool ldd_bottom_up(const DevScalars* sc, int cur, int64_t n, int64_t m) {
  const long long fe = sc->ldd_fe[cur];
  const long long mu = (long long)m - sc->ldd_seen - fe;
  return fe * kLddAlpha > mu && fe * kLddGamma > (long long)n;
}

// Adds the block's degree sums to an LDD frontier accumulator: one atomic
// per block (same-address atomics from every wave serialize at one L2
// channel and cost a late grid round hundreds of microseconds).  Called by
// every thread of the block.
__device__ __forceinline__ void ldd_add_edges(long long x, long long* acc) {
  __shared__ long long red[kFBlock / kWave];
  x = wave_sum(x);
  if (lane_id() == 0) red[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < kFBlock / kWave; ++w) t += red[w];
    if (t) atomicAdd((unsigned long long*)acc, (unsigned long long)t);
  }
}

// One LDD round (LDD = true) or frontier expansion.  Top-down: the frontier
// queue's rows, wave-balanced, rows above kHeavyFrontier left to the grid
// kernel; a claimed vertex joins its claimer's cluster.  Bottom-up (LDD,
// when ldd_bottom_up holds): every unvisited vertex scans its row for a
// neighbour stamped with this round (a member of the frontier) and joins
// that neighbour's cluster; lanes map to consecutive vertices, so each
// half-wave owns one bitmap word and writes it without atomics.  Claimed
// vertices get stamp round + 1 and go to the next queue; their degrees are
// added to the next frontier's edge count.
template <bool LDD, typename I>
__global__ void __launch_bounds__(kFBlock) k_expand(const int32_t* __restrict__ qin, const uint32_t* cnt_in,
                                                    int32_t* qout, uint32_t* cnt_out, const I* __restrict__ off,
                                                    const int32_t* __restrict__ adj, uint32_t* vis, uint32_t* fn,
                                                    int32_t* P, int32_t* heavy, long long* hp,
                                                    unsigned long long* pack, int2* tree, int32_t* stamp,
                                                    int32_t round, int64_t n, int64_t m, DevScalars* sc, int cur) {
  constexpr int W = kFBlock / kWave;
  __shared__ int32_t qbuf[W][kWaveQCap];
  __shared__ int32_t tpre[W][kWave + 1];
  __shared__ int64_t tbeg[W][kWave];
  __shared__ int32_t tlab[W][kWave];
  __shared__ int32_t tu[W][kWave];
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  WaveQ q{qbuf[wv], 0};
  long long added = 0;
  if (LDD && ldd_bottom_up(sc, cur, n, m)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) ++sc->bu_rounds;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
      const int64_t v = base + threadIdx.x;
      bool found = false;
      if (v < n && !bit_get(vis, v)) {
        const int64_t b = (int64_t)off[v];
        const int64_t e = (int64_t)off[v + 1];
        for (int64_t j = b; j < e; ++j) {
          const int32_t x = adj[j];
          if (stamp[x] == round) {
            found = true;
            P[v] = P[x];
            stamp[v] = round + 1;
            if (tree) tree[v] = make_int2(x, (int32_t)v);
            added += e - b;
            break;
          }
        }
      }
      // base is a multiple of 256: lanes 0-31 and 32-63 each cover one word
      const uint64_t bits = __ballot(found);
      if ((lane & 31) == 0 && v < n) {
        const uint32_t wbits = (uint32_t)(bits >> (lane & 32));
        if (wbits) vis[v >> 5] |= wbits;
      }
      wq_push(q, found, (int32_t)v, qout, cnt_out);
    }
    wq_flush(q, qout, cnt_out);
    ldd_add_edges(added, &sc->ldd_fe[cur ^ 1]);
    return;
  }
  const int64_t cnt = *cnt_in;
  const int64_t tiles = (cnt + kWave - 1) / kWave;
  const int64_t waves = (int64_t)gridDim.x * W;
  for (int64_t tile = blockIdx.x * (int64_t)W + wv; tile < tiles; tile += waves) {
    const int64_t idx = tile * kWave + lane;
    int32_t u = 0;
    int64_t b = 0, d = 0;
    if (idx < cnt) {
      u = qin[idx];
      b = (int64_t)off[u];
      d = (int64_t)off[u + 1] - b;
    }
    const bool heavy_row = d > kHeavyFrontier;
    heavy_reserve(heavy_row, u, d, heavy, hp, pack);
    if (heavy_row) d = 0;
    // exclusive scan of the row lengths across the wave
    int32_t inc = (int32_t)d;
    for (int o = 1; o < kWave; o <<= 1) {
      const int32_t y = __shfl_up(inc, o, kWave);
      if (lane >= o) inc += y;
    }
    const int32_t total = __shfl(inc, kWave - 1, kWave);
    tpre[wv][lane] = inc - (int32_t)d;
    if (lane == kWave - 1) tpre[wv][kWave] = total;
    tbeg[wv][lane] = b;
    tu[wv][lane] = u;
    if (LDD) tlab[wv][lane] = (idx < cnt) ? P[u] : 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int32_t e0 = 0; e0 < total; e0 += kWave) {
      const int32_t e = e0 + lane;
      bool got = false;
      int32_t w = 0;
      if (e < total) {
        int lo = 0, hi = kWave - 1;  // last row whose start <= e
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (tpre[wv][mid] <= e) lo = mid;
          else hi = mid - 1;
        }
        w = adj[tbeg[wv][lo] + (e - tpre[wv][lo])];
        got = bit_claim(vis, w);
        if (got) {
          if (LDD) {
            P[w] = tlab[wv][lo];
            stamp[w] = round + 1;
            added += (long long)off[w + 1] - (long long)off[w];
          } else {
            aor(fn + (w >> 5), 1u << (w & 31));
          }
          if (tree) tree[w] = make_int2(tu[wv][lo], w);
        }
      }
      wq_push(q, got, w, qout, cnt_out);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  wq_flush(q, qout, cnt_out);
  if (LDD) ldd_add_edges(added, &sc->ldd_fe[cur ^ 1]);
}

// Rows of heavy frontier vertices, spread evenly over the whole grid.
template <bool LDD, typename I>
__global__ void __launch_bounds__(kFBlock) k_expand_heavy(const int32_t* __restrict__ heavy,
                                                          const unsigned long long* pack,
                                                          const long long* __restrict__ hp, const I* __restrict__ off,
                                                          const int32_t* __restrict__ adj, uint32_t* vis,
                                                          uint32_t* fn, int32_t* P, int32_t* qout,
                                                          uint32_t* cnt_out, int2* tree, int32_t* stamp,
                                                          int32_t round, int64_t n, int64_t m, DevScalars* sc,
                                                          int cur) {
  __shared__ int32_t qbuf[kFBlock / kWave][kWaveQCap];
  WaveQ q{qbuf[threadIdx.x / kWave], 0};
  if (LDD && ldd_bottom_up(sc, cur, n, m)) return;  // the round runs bottom-up
  long long added = 0;
  const unsigned long long pk = *pack;
  const int64_t c = (int64_t)(pk >> kPackShift);
  if (c == 0) return;
  const long long T = (long long)(pk & kPackEdges);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (long long base = blockIdx.x * (int64_t)blockDim.x; base < T; base += stride) {
    const long long e = base + threadIdx.x;
    const long long e0 = base + (threadIdx.x / kWave) * kWave;
    bool got = false;
    int32_t w = 0;
    if (e < T) {
      const int64_t i = heavy_owner_tile(hp, c, e0, e);
      const int32_t u = heavy[i];
      w = adj[(int64_t)off[u] + (e - hp[i])];
      got = bit_claim(vis, w);
      if (got) {
        if (LDD) {
          P[w] = P[u];
          stamp[w] = round + 1;
          added += (long long)off[w + 1] - (long long)off[w];
        } else {
          aor(fn + (w >> 5), 1u << (w & 31));
        }
        if (tree) tree[w] = make_int2(u, w);
      }
    }
    wq_push(q, got, w, qout, cnt_out);
  }
  wq_flush(q, qout, cnt_out);
  if (LDD) ldd_add_edges(added, &sc->ldd_fe[cur ^ 1]);
}

// Minimum reached vertex = lowest set bit of the visited bitmap (one atomic
// per block; the grid is kept small).
__global__ void __launch_bounds__(kFBlock) k_bitmap_min(const uint32_t* __restrict__ vis, int64_t words,
                                                        DevScalars* sc) {
  __shared__ int32_t red[kFBlock / kWave];
  int32_t best = 0x7fffffff;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += stride) {
    const uint32_t w = vis[i];
    if (w) {
      const int32_t x = (int32_t)(i * 32 + __ffs(w) - 1);
      best = x < best ? x : best;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t y = __shfl_xor(best, o, kWave);
    best = y < best ? y : best;
  }
  if (lane_id() == 0) red[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kFBlock / kWave; ++w) best = red[w] < best ? red[w] : best;
    if (best != 0x7fffffff) atomicMin(&sc->bfs_min, best);
  }
}

__global__ void k_label_reached(int64_t n, const uint32_t* __restrict__ vis, const DevScalars* sc, int32_t* P) {
  const int32_t mn = sc->bfs_min;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride)
    if (bit_get(vis, v)) P[v] = mn;
}

// One BFS from `source` (every level device-driven, see above).
template <typename I>
cc_status bfs_probe(StaticArgs& a, int32_t source, int level_cap, int64_t* reached_out, int32_t* levels_out) {
  const int64_t n = a.n, m = a.m;
  const int64_t words = (n + 31) / 32;
  const size_t bw = align256((size_t)words * 4);
  uint32_t* vis = (uint32_t*)(a.ws + a.L.bits);
  uint32_t* fa = (uint32_t*)(a.ws + a.L.bits + bw);
  uint32_t* fb = (uint32_t*)(a.ws + a.L.bits + 2 * bw);
  int32_t* q[2] = {(int32_t*)(a.ws + a.L.queue), (int32_t*)(a.ws + a.L.queue + align256((size_t)n * 4))};
  long long* fpart = (long long*)(a.ws + a.L.hist);   // kBfsParts entries (the LDD histogram area)
  const I* off = (const I*)a.off;
  DevScalars* sc = a.ctx->dev;
  if (m >= (int64_t(1) << kPackShift))
    return fail(CC_EINVAL, "BFS sampling takes m < 2^%d adjacency entries (m=%lld)", kPackShift, (long long)m);
  cc_status st = count_heavy<I>(a);
  if (st != CC_OK) return st;
  const bool heavy = a.heavy_vertices > 0;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(3 * bw / 4, kFBlock, 4096)), dim3(kFBlock), 0, a.s, vis,
                     (int64_t)(3 * bw / 4), 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(16), dim3(kFBlock), 0, a.s, (uint32_t*)fpart, (int64_t)kBfsParts * 2, 0u);
  hipLaunchKernelGGL(k_bfs_start<I>, dim3(1), dim3(1), 0, a.s, source, off, vis, fa, q[0], sc);
  CC_LAUNCH_CHECK();
  const unsigned gb = grid_for(words, kFBlock, 1024);
  const unsigned gs = grid_for(n, kFBlock, kBfsStepBlocks);
  const unsigned gh = kBfsParts - kBfsStepBlocks;
  uint32_t* fc = fa;
  uint32_t* fn = fb;
  int cur = 0;
  int64_t launched = 0;
  int batch = 2;
  int slot = 0;
  bool have_prev = false;
  hipEvent_t* ev = a.ctx->ring_ev;
  struct Snap {
    uint32_t mode;
    int32_t level;
    long long reached;
  };
  Snap* ring = (Snap*)a.ctx->ring_host;
  Snap fin{kBfsTopDown, 0, 1};
  cc_status result = CC_OK;
  while (true) {
    for (int j = 0; j < batch; ++j) {
      hipLaunchKernelGGL(k_bfs_begin, dim3(gb), dim3(kFBlock), 0, a.s, words, fn, sc, cur, (const long long*)fpart, n,
                         m, level_cap);
      hipLaunchKernelGGL(k_bfs_step<I>, dim3(gs), dim3(kFBlock), 0, a.s, n, off, a.adj, vis, (const uint32_t*)fc, fn,
                         (const int32_t*)q[cur], &sc->qcount[cur], q[cur ^ 1], &sc->qcount[cur ^ 1], a.heavy,
                         a.hp, sc, fpart, a.tree_e);
      if (heavy)
        hipLaunchKernelGGL(k_bfs_heavy<I>, dim3(gh), dim3(kFBlock), 0, a.s, (const int32_t*)a.heavy,
                           (const long long*)a.hp, off, a.adj, vis, fn, q[cur ^ 1], &sc->qcount[cur ^ 1],
                           (const DevScalars*)sc, fpart, a.tree_e);
      uint32_t* t2 = fc;
      fc = fn;
      fn = t2;
      cur ^= 1;
      ++launched;
    }
    CC_LAUNCH_CHECK();
    CC_HIP(hipMemcpyAsync(&ring[slot], &sc->bfs_mode, sizeof(Snap), hipMemcpyDeviceToHost, a.s));
    CC_HIP(hipEventRecord(ev[slot], a.s));
    if (have_prev) {
      CC_HIP(hipEventSynchronize(ev[slot ^ 1]));
      const Snap sn = ring[slot ^ 1];
      if (sn.mode == kBfsDone) {
        fin = sn;
        break;
      }
      if (a.ctx->round_limit > 0 && sn.level >= a.ctx->round_limit) {
        result = fail(CC_ELIVELOCK, "BFS reached the context's round limit (%d)", a.ctx->round_limit);
        break;
      }
      // a search expands at most n levels; the host runs at most two
      // batches (<= 64 levels) ahead of the snapshot it reads
      if (sn.level > n + 1 || launched > n + 2 + 2 * 32) {
        result = fail(CC_ELIVELOCK, "BFS exceeded n levels");
        break;
      }
    }
    have_prev = true;
    slot ^= 1;
    batch = batch < 32 ? 2 * batch : 32;
  }
  // the batch queued after the finishing snapshot does nothing; wait for it
  CC_HIP(hipStreamSynchronize(a.s));
  if (result != CC_OK) return result;
  *reached_out = fin.reached;
  *levels_out = fin.level;
  return CC_OK;
}

template <typename I>
cc_status sample_bfs(StaticArgs& a) {
  const int64_t n = a.n;
  const int64_t words = (n + 31) / 32;
  uint32_t* vis = (uint32_t*)(a.ws + a.L.bits);
  DevScalars* sc = a.ctx->dev;
  const uint64_t key = sm_out(a.v->seed, kTagBfs);
  a.sample_success = -1;
  a.sample_rounds = 0;
  for (int t = 0; t < a.v->bfs_tries; ++t) {
    const int32_t s = (int32_t)(sm_out(key, (uint64_t)t) % (uint64_t)n);
    int64_t reached = 0;
    int32_t levels = 0;
    cc_status st = bfs_probe<I>(a, s, 0, &reached, &levels);
    if (st != CC_OK) return st;
    a.sample_rounds += levels;
    if (10 * reached <= n && a.tree_e)   // a failed try's tree edges are not a sample
      hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(2 * n, kFBlock, 4096)), dim3(kFBlock), 0, a.s,
                         (uint32_t*)a.tree_e, 2 * n, 0xffffffffu);
    if (10 * reached > n) {
      hipLaunchKernelGGL(k_bitmap_min, dim3(grid_for(words, kFBlock, 256)), dim3(kFBlock), 0, a.s, vis, words, sc);
      hipLaunchKernelGGL(k_label_reached, dim3(grid_for(n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, n,
                         (const uint32_t*)vis, (const DevScalars*)sc, a.P);
      CC_LAUNCH_CHECK();
      a.sample_success = t;
      return CC_OK;
    }
  }
  return CC_OK;  // every try failed: identity labelling, nothing skipped
}

// ---- LDD --------------------------------------------------------------------

__device__ __forceinline__ uint32_t ldd_u24(uint64_t key, int64_t v) { return (uint32_t)(sm_out(key, (uint64_t)v) >> 40); }
__device__ __forceinline__ float ldd_delta(uint32_t u24, float beta) {
  // U in (0, 1): (u24 + 0.5) / 2^24; delta = -ln(U) / beta
  return -logf(((float)u24 + 0.5f) * (1.0f / 16777216.0f)) / beta;
}

// Minimum draw (largest shift) and min-member scratch init; one atomic per
// block (the grid is kept small).
constexpr int kLddGrid = 256;

__global__ void __launch_bounds__(kFBlock) k_ldd_prep(int64_t n, uint64_t key, int32_t* mn, DevScalars* sc) {
  __shared__ uint32_t red[kFBlock / kWave];
  uint32_t best = 0xffffffffu;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const uint32_t u = ldd_u24(key, v);
    best = u < best ? u : best;
    mn[v] = (int32_t)v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t y = __shfl_xor(best, o, kWave);
    best = y < best ? y : best;
  }
  if (lane_id() == 0) red[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kFBlock / kWave; ++w) best = red[w] < best ? red[w] : best;
    atomicMin(&sc->pad[0], best);
    if (blockIdx.x == 0) sc->ldd_fe[0] = sc->ldd_fe[1] = sc->ldd_seen = 0;
  }
}

constexpr int kLddMaxRounds = 4096;

// Start-round histogram: per-block LDS counts, added once per block.
__global__ void k_ldd_hist(int64_t n, uint64_t key, float beta, const DevScalars* sc, uint32_t* hist) {
  __shared__ uint32_t h[kLddMaxRounds];
  for (int i = threadIdx.x; i < kLddMaxRounds; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const float dmax = ldd_delta(sc->pad[0], beta);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const float d = ldd_delta(ldd_u24(key, v), beta);
    int r = (int)floorf(dmax - d);
    r = r < 0 ? 0 : (r >= kLddMaxRounds ? kLddMaxRounds - 1 : r);
    atomicAdd(&h[r], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kLddMaxRounds; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Vertices [lo, hi) wake: the unvisited ones become cluster centres
// (stamped with the round).  Lanes map to consecutive vertices from a
// 32-aligned start, so each half-wave owns one bitmap word and writes it
// without atomics.  Only centres with an edge join the frontier (an
// isolated centre has nothing to expand); their degrees join its edge
// count.  Block 0 also resets the round's output queue (queue `nxt`), its
// edge count (after adding the last frontier's to the expanded total) and
// the heavy list.
template <typename I>
__global__ void __launch_bounds__(kFBlock) k_ldd_wake(int64_t lo, int64_t hi, const I* __restrict__ off,
                                                      uint32_t* vis, int32_t* P, int32_t* q, uint32_t* cnt,
                                                      DevScalars* sc, int nxt, int32_t* stamp, int32_t round) {
  __shared__ int32_t qbuf[kFBlock / kWave][kWaveQCap];
  WaveQ wq{qbuf[threadIdx.x / kWave], 0};
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->qcount[nxt] = 0;
    sc->heavy_pack = 0ull;
    sc->ldd_seen += sc->ldd_fe[nxt];
    sc->ldd_fe[nxt] = 0;
  }
  long long added = 0;
  const int lane = lane_id();
  const int64_t lo32 = lo & ~(int64_t)31;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = lo32 + blockIdx.x * (int64_t)blockDim.x; base < hi; base += stride) {
    const int64_t v = base + threadIdx.x;
    const bool got = v >= lo && v < hi && !bit_get(vis, v);
    if (got) {
      P[v] = (int32_t)v;
      stamp[v] = round;
    }
    const uint64_t bits = __ballot(got);
    if ((lane & 31) == 0) {
      const uint32_t wbits = (uint32_t)(bits >> (lane & 32));
      if (wbits) vis[v >> 5] |= wbits;
    }
    const int64_t d = got ? (int64_t)off[v + 1] - (int64_t)off[v] : 0;
    added += d;
    wq_push(wq, d > 0, (int32_t)v, q, cnt);
  }
  wq_flush(wq, q, cnt);
  ldd_add_edges(added, &sc->ldd_fe[nxt ^ 1]);
}

// Minimum member of every cluster.  mn[c] starts at c, so only members with
// a smaller id than their centre can lower it (after a plain read shows they
// would); clusters whose minimum moved are marked in `moved`, so the relabel
// reads mn only for those.
__global__ void __launch_bounds__(kFBlock) k_min_member(int64_t n, const int32_t* __restrict__ P, int32_t* mn,
                                                        uint32_t* moved) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t c = P[v];
    if ((int32_t)v < c && (int32_t)v < ld(mn + c)) {
      amin(mn + c, (int32_t)v);
      if (!bit_get(moved, c)) aor(moved + (c >> 5), 1u << (c & 31));
    }
  }
}

__global__ void k_relabel(int64_t n, int32_t* P, const int32_t* __restrict__ mn, const uint32_t* __restrict__ moved) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t c = P[v];
    if (bit_get(moved, c)) P[v] = mn[c];
  }
}

template <typename I>
cc_status sample_ldd(StaticArgs& a) {
  const int64_t n = a.n;
  const int64_t words = (n + 31) / 32;
  uint32_t* vis = (uint32_t*)(a.ws + a.L.bits);
  int32_t* q[2] = {(int32_t*)(a.ws + a.L.queue), (int32_t*)(a.ws + a.L.queue + align256((size_t)n * 4))};
  uint32_t* hist = (uint32_t*)(a.ws + a.L.hist);
  int32_t* mn = a.cand;  // candidates are only compacted after sampling
  const I* off = (const I*)a.off;
  DevScalars* sc = a.ctx->dev;
  const uint64_t key = sm_out(a.v->seed, kTagLdd);
  const float beta = a.v->ldd_beta;
  if (a.m >= (int64_t(1) << kPackShift))
    return fail(CC_EINVAL, "LDD sampling takes m < 2^%d adjacency entries (m=%lld)", kPackShift, (long long)a.m);

  cc_status st = count_heavy<I>(a);
  if (st != CC_OK) return st;
  const bool heavy = a.heavy_vertices > 0;
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, a.s, &sc->pad[0], 0xffffffffu);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words, kFBlock, 4096)), dim3(kFBlock), 0, a.s, vis, words, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(16), dim3(kFBlock), 0, a.s, hist, (int64_t)kLddMaxRounds, 0u);
  // the round each vertex entered a frontier (-1: not yet); the wave-bin
  // candidate array is free until the compaction
  int32_t* stamp = a.big;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, (uint32_t*)stamp, n,
                     0xffffffffu);
  hipLaunchKernelGGL(k_ldd_prep, dim3(grid_for(n, kFBlock, kLddGrid)), dim3(kFBlock), 0, a.s, n, key, mn, sc);
  hipLaunchKernelGGL(k_ldd_hist, dim3(grid_for(n, kFBlock, kLddGrid)), dim3(kFBlock), 0, a.s, n, key, beta,
                     (const DevScalars*)sc, hist);
  CC_LAUNCH_CHECK();
  std::vector<uint32_t> h(kLddMaxRounds);
  CC_HIP(hipMemcpyAsync(h.data(), hist, kLddMaxRounds * 4, hipMemcpyDeviceToHost, a.s));
  CC_HIP(hipStreamSynchronize(a.s));
  int last = 0;
  for (int r = 0; r < kLddMaxRounds; ++r)
    if (h[r]) last = r;
  // both queue counters start at zero; each wake resets the other one
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, a.s, &sc->qcount[0], 0u);
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, a.s, &sc->qcount[1], 0u);
  int64_t lo = 0, S = 0;
  int cur = 0;
  for (int r = 0; r <= last; ++r) {
    S += h[r];
    const int64_t hi = (r == last) ? n : S;
    const int nxt = cur ^ 1;
    hipLaunchKernelGGL(k_ldd_wake<I>, dim3(grid_for(hi > lo ? hi - (lo & ~(int64_t)31) : 1, kFBlock, 1024)),
                       dim3(kFBlock), 0, a.s, lo, hi, off, vis, a.P, q[cur], &sc->qcount[cur], sc, nxt, stamp, r);
    lo = hi > lo ? hi : lo;
    hipLaunchKernelGGL((k_expand<true, I>), dim3(grid_for(n, kFBlock, 2048)), dim3(kFBlock), 0, a.s, q[cur],
                       &sc->qcount[cur], q[nxt], &sc->qcount[nxt], off, a.adj, vis, (uint32_t*)nullptr, a.P,
                       a.heavy, a.hp, &sc->heavy_pack, a.tree_e, stamp, r, n, a.m, sc, cur);
    if (heavy)
      hipLaunchKernelGGL((k_expand_heavy<true, I>), dim3(2048), dim3(kFBlock), 0, a.s, (const int32_t*)a.heavy,
                         (const unsigned long long*)&sc->heavy_pack, (const long long*)a.hp, off, a.adj, vis,
                         (uint32_t*)nullptr, a.P, q[nxt], &sc->qcount[nxt], a.tree_e, stamp, r, n, a.m, sc, cur);
    CC_LAUNCH_CHECK();
    cur = nxt;
    ++a.sample_rounds;
  }
  // After the last wake every vertex is visited; the last expansion claimed
  // nothing new.  Relabel each cluster to its minimum member.
  uint32_t* moved = (uint32_t*)(a.ws + a.L.bits + align256((size_t)words * 4));   // second bitmap
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words, kFBlock, 4096)), dim3(kFBlock), 0, a.s, moved, words, 0u);
  hipLaunchKernelGGL(k_min_member, dim3(grid_for(n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, n, (const int32_t*)a.P,
                     mn, moved);
  hipLaunchKernelGGL(k_relabel, dim3(grid_for(n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, n, a.P,
                     (const int32_t*)mn, (const uint32_t*)moved);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

template cc_status bfs_probe<int32_t>(StaticArgs&, int32_t, int, int64_t*, int32_t*);
template cc_status bfs_probe<int64_t>(StaticArgs&, int32_t, int, int64_t*, int32_t*);
template cc_status sample_bfs<int32_t>(StaticArgs&);
template cc_status sample_bfs<int64_t>(StaticArgs&);
template cc_status sample_ldd<int32_t>(StaticArgs&);
template cc_status sample_ldd<int64_t>(StaticArgs&);

}  // namespace cc
