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

template <typename I>
__global__ void k_bfs_start(int32_t s, const I* off, uint32_t* vis, uint32_t* fc, int32_t* q0, DevScalars* sc) {
  vis[s >> 5] |= 1u << (s & 31);
  fc[s >> 5] |= 1u << (s & 31);
  q0[0] = s;
  sc->qcount[0] = 1;
  sc->qcount[1] = 0;
  sc->frontier_edges = (long long)off[s + 1] - (long long)off[s];
}

// Prepares the next level: clears the next-frontier bitmap and its counter.
__global__ void k_bfs_level_reset(uint32_t* fn, int64_t words, DevScalars* sc, int nxt) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i == 0) {
    sc->qcount[nxt] = 0;
    sc->frontier_edges = 0;
    sc->hcount = 0;
  }
  for (; i < words; i += stride) fn[i] = 0u;
}

// Frontier expansion (BFS top-down step, LDD cluster growth), load-balanced
// within each wave: a wave takes 64 frontier vertices, concatenates their
// rows (exclusive scan of the degrees across lanes) and walks the joint edge
// list 64 edges at a time; each lane finds the row of its edge by a binary
// search over the 64 row starts in LDS.  Rows above kHeavyFrontier are
// deferred to the grid kernel.  Claimed vertices go through a wave-private
// LDS buffer, so the output queue's counter is bumped once per flush.
template <bool LDD, typename I>
__global__ void __launch_bounds__(kFBlock) k_expand(const int32_t* __restrict__ qin, const uint32_t* cnt_in,
                                                    int32_t* qout, uint32_t* cnt_out, const I* __restrict__ off,
                                                    const int32_t* __restrict__ adj, uint32_t* vis, uint32_t* fn,
                                                    int32_t* P, int32_t* heavy, int32_t* hcount) {
  constexpr int W = kFBlock / kWave;
  __shared__ int32_t qbuf[W][kWaveQCap];
  __shared__ int32_t tpre[W][kWave + 1];
  __shared__ int64_t tbeg[W][kWave];
  __shared__ int32_t tlab[W][kWave];
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  WaveQ q{qbuf[wv], 0};
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
    wave_append(heavy_row, u, heavy, (uint32_t*)hcount);  // rare: one atomic per wave with a heavy row
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
          if (LDD) P[w] = tlab[wv][lo];
          else aor(fn + (w >> 5), 1u << (w & 31));
        }
      }
      wq_push(q, got, w, qout, cnt_out);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  wq_flush(q, qout, cnt_out);
}

// Bottom-up step: every unvisited vertex looks for a neighbour in the
// current frontier bitmap and stops at the first one.
template <typename I>
__global__ void __launch_bounds__(kFBlock) k_bfs_bu(int64_t n, const I* __restrict__ off,
                                                    const int32_t* __restrict__ adj, uint32_t* vis,
                                                    const uint32_t* __restrict__ fc, uint32_t* fn, int32_t* qout,
                                                    uint32_t* cnt_out) {
  __shared__ int32_t qbuf[kFBlock / kWave][kWaveQCap];
  WaveQ q{qbuf[threadIdx.x / kWave], 0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    bool found = false;
    if (v < n && !bit_get(vis, v)) {
      const int64_t e = (int64_t)off[v + 1];
      for (int64_t j = (int64_t)off[v]; j < e; ++j)
        if (bit_get(fc, adj[j])) {
          found = true;
          break;
        }
    }
    if (found) {
      aor(vis + (v >> 5), 1u << (v & 31));
      aor(fn + (v >> 5), 1u << (v & 31));
    }
    wq_push(q, found, (int32_t)v, qout, cnt_out);
  }
  wq_flush(q, qout, cnt_out);
}

// Rows of heavy frontier vertices, spread evenly over the whole grid.
template <bool LDD, typename I>
__global__ void __launch_bounds__(kFBlock) k_expand_heavy(const int32_t* __restrict__ heavy, const int32_t* hcount,
                                                          const long long* __restrict__ hp, const I* __restrict__ off,
                                                          const int32_t* __restrict__ adj, uint32_t* vis,
                                                          uint32_t* fn, int32_t* P, int32_t* qout,
                                                          uint32_t* cnt_out) {
  __shared__ int32_t qbuf[kFBlock / kWave][kWaveQCap];
  WaveQ q{qbuf[threadIdx.x / kWave], 0};
  const int64_t c = *hcount;
  if (c == 0) return;
  const long long T = hp[c];
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
        if (LDD) P[w] = P[u];
        else aor(fn + (w >> 5), 1u << (w & 31));
      }
    }
    wq_push(q, got, w, qout, cnt_out);
  }
  wq_flush(q, qout, cnt_out);
}

__global__ void k_round_reset(DevScalars* sc, int nxt) {
  sc->qcount[nxt] = 0;
  sc->hcount = 0;
}

template <typename I>
__global__ void k_sum_degrees(const int32_t* __restrict__ q, const uint32_t* cnt, const I* __restrict__ off,
                              DevScalars* sc) {
  const int64_t c = *cnt;
  long long s = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += stride) {
    const int32_t u = q[i];
    s += (long long)off[u + 1] - (long long)off[u];
  }
  s = wave_sum(s);
  if (lane_id() == 0 && s) add64(&sc->frontier_edges, s);
}

// Minimum reached vertex = lowest set bit of the visited bitmap.
__global__ void k_bitmap_min(const uint32_t* __restrict__ vis, int64_t words, DevScalars* sc) {
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
  if (lane_id() == 0 && best != 0x7fffffff) atomicMin(&sc->bfs_min, best);
}

__global__ void k_label_reached(int64_t n, const uint32_t* __restrict__ vis, const DevScalars* sc, int32_t* P) {
  const int32_t mn = sc->bfs_min;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride)
    if (bit_get(vis, v)) P[v] = mn;
}

// One direction-optimizing BFS from `source` into the visited bitmap.
template <typename I>
cc_status bfs_probe(StaticArgs& a, int32_t source, int level_cap, int64_t* reached_out, int32_t* levels_out) {
  const int64_t n = a.n, m = a.m;
  const int64_t words = (n + 31) / 32;
  const size_t bw = align256((size_t)words * 4);
  uint32_t* vis = (uint32_t*)(a.ws + a.L.bits);
  uint32_t* fa = (uint32_t*)(a.ws + a.L.bits + bw);
  uint32_t* fb = (uint32_t*)(a.ws + a.L.bits + 2 * bw);
  int32_t* q[2] = {(int32_t*)(a.ws + a.L.queue), (int32_t*)(a.ws + a.L.queue + align256((size_t)n * 4))};
  const I* off = (const I*)a.off;
  DevScalars* sc = a.ctx->dev;
  const double alpha = 15.0, beta = 18.0;  // Beamer's direction-switch constants
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(3 * bw / 4, kFBlock, 4096)), dim3(kFBlock), 0, a.s, vis,
                     (int64_t)(3 * bw / 4), 0u);
  hipLaunchKernelGGL(k_bfs_start<I>, dim3(1), dim3(1), 0, a.s, source, off, vis, fa, q[0], sc);
  CC_LAUNCH_CHECK();
  cc_status st = pull_scalars(a);
  if (st != CC_OK) return st;
  int64_t nf = 1, mf = a.ctx->host->frontier_edges, seen_edges = mf, reached = 1;
  bool top_down = true;
  int cur = 0;
  int32_t levels = 0;
  uint32_t* fc = fa;
  uint32_t* fn = fb;
  for (int level = 0; nf > 0 && (level_cap <= 0 || level < level_cap); ++level) {
    if (level > n + 1) return fail(CC_ELIVELOCK, "BFS exceeded n levels");
    if (a.ctx->round_limit > 0 && level >= a.ctx->round_limit)
      return fail(CC_ELIVELOCK, "BFS reached the context's round limit (%d)", a.ctx->round_limit);
    if (top_down && (double)mf > (double)(m - seen_edges + mf) / alpha) top_down = false;
    else if (!top_down && (double)nf < (double)n / beta) top_down = true;
    const int nxt = cur ^ 1;
    hipLaunchKernelGGL(k_bfs_level_reset, dim3(grid_for(words, kFBlock, 4096)), dim3(kFBlock), 0, a.s, fn, words,
                       sc, nxt);
    if (top_down) {
      hipLaunchKernelGGL((k_expand<false, I>), dim3(grid_for(nf * kWave / kWave, kFBlock, 2048)), dim3(kFBlock), 0,
                         a.s, q[cur], &sc->qcount[cur], q[nxt], &sc->qcount[nxt], off, a.adj, vis, fn,
                         (int32_t*)nullptr, a.heavy, &sc->hcount);
      heavy_prefix<I>(a.s, a.heavy, (const int32_t*)&sc->hcount, a.hcap, off, a.tsum, a.hp);
      hipLaunchKernelGGL((k_expand_heavy<false, I>), dim3(2048), dim3(kFBlock), 0, a.s, (const int32_t*)a.heavy,
                         (const int32_t*)&sc->hcount, (const long long*)a.hp, off, a.adj, vis, fn,
                         (int32_t*)nullptr, q[nxt], &sc->qcount[nxt]);
    } else {
      hipLaunchKernelGGL(k_bfs_bu<I>, dim3(grid_for(n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, n, off, a.adj, vis,
                         fc, fn, q[nxt], &sc->qcount[nxt]);
    }
    hipLaunchKernelGGL(k_sum_degrees<I>, dim3(grid_for(n, kFBlock, 1024)), dim3(kFBlock), 0, a.s, q[nxt],
                       &sc->qcount[nxt], off, sc);
    CC_LAUNCH_CHECK();
    st = pull_scalars(a);
    if (st != CC_OK) return st;
    nf = a.ctx->host->qcount[nxt];
    mf = a.ctx->host->frontier_edges;
    seen_edges += mf;
    reached += nf;
    uint32_t* t2 = fc;
    fc = fn;
    fn = t2;
    cur = nxt;
    ++levels;
  }
  *reached_out = reached;
  *levels_out = levels;
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
    if (10 * reached > n) {
      hipLaunchKernelGGL(k_bitmap_min, dim3(grid_for(words, kFBlock, 1024)), dim3(kFBlock), 0, a.s, vis, words, sc);
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

// Minimum draw (largest shift) and min-member scratch init.
__global__ void k_ldd_prep(int64_t n, uint64_t key, int32_t* mn, DevScalars* sc) {
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
  if (lane_id() == 0) atomicMin(&sc->pad[0], best);
}

constexpr int kLddMaxRounds = 4096;

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

// Vertices [lo, hi) wake: the unvisited ones become cluster centres.
__global__ void __launch_bounds__(kFBlock) k_ldd_wake(int64_t lo, int64_t hi, uint32_t* vis, int32_t* P, int32_t* q,
                                                      uint32_t* cnt) {
  __shared__ int32_t qbuf[kFBlock / kWave][kWaveQCap];
  WaveQ wq{qbuf[threadIdx.x / kWave], 0};
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = lo + blockIdx.x * (int64_t)blockDim.x; base < hi; base += stride) {
    const int64_t v = base + threadIdx.x;
    bool got = false;
    if (v < hi) {
      got = bit_claim(vis, v);
      if (got) P[v] = (int32_t)v;
    }
    wq_push(wq, got, (int32_t)v, q, cnt);
  }
  wq_flush(wq, q, cnt);
}

__global__ void k_min_member(int64_t n, const int32_t* __restrict__ P, int32_t* mn) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t c = P[v];
    if ((int32_t)v < ld(mn + c)) amin(mn + c, (int32_t)v);
  }
}

__global__ void k_relabel(int64_t n, int32_t* P, const int32_t* __restrict__ mn) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) P[v] = mn[P[v]];
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

  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, a.s, &sc->pad[0], 0xffffffffu);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words, kFBlock, 4096)), dim3(kFBlock), 0, a.s, vis, words, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(16), dim3(kFBlock), 0, a.s, hist, (int64_t)kLddMaxRounds, 0u);
  hipLaunchKernelGGL(k_ldd_prep, dim3(grid_for(n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, n, key, mn, sc);
  hipLaunchKernelGGL(k_ldd_hist, dim3(grid_for(n, kFBlock, 2048)), dim3(kFBlock), 0, a.s, n, key, beta,
                     (const DevScalars*)sc, hist);
  CC_LAUNCH_CHECK();
  std::vector<uint32_t> h(kLddMaxRounds);
  CC_HIP(hipMemcpyAsync(h.data(), hist, kLddMaxRounds * 4, hipMemcpyDeviceToHost, a.s));
  CC_HIP(hipStreamSynchronize(a.s));
  int last = 0;
  for (int r = 0; r < kLddMaxRounds; ++r)
    if (h[r]) last = r;
  // reset both queue counters
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, a.s, &sc->qcount[0], 0u);
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, a.s, &sc->qcount[1], 0u);
  int64_t lo = 0, S = 0;
  int cur = 0;
  for (int r = 0; r <= last; ++r) {
    S += h[r];
    const int64_t hi = (r == last) ? n : S;
    if (hi > lo)
      hipLaunchKernelGGL(k_ldd_wake, dim3(grid_for(hi - lo, kFBlock, 4096)), dim3(kFBlock), 0, a.s, lo, hi, vis, a.P,
                         q[cur], &sc->qcount[cur]);
    lo = hi;
    const int nxt = cur ^ 1;
    hipLaunchKernelGGL(k_round_reset, dim3(1), dim3(1), 0, a.s, sc, nxt);
    hipLaunchKernelGGL((k_expand<true, I>), dim3(grid_for(n, kFBlock, 2048)), dim3(kFBlock), 0, a.s, q[cur],
                       &sc->qcount[cur], q[nxt], &sc->qcount[nxt], off, a.adj, vis, (uint32_t*)nullptr, a.P,
                       a.heavy, &sc->hcount);
    heavy_prefix<I>(a.s, a.heavy, (const int32_t*)&sc->hcount, a.hcap, off, a.tsum, a.hp);
    hipLaunchKernelGGL((k_expand_heavy<true, I>), dim3(2048), dim3(kFBlock), 0, a.s, (const int32_t*)a.heavy,
                       (const int32_t*)&sc->hcount, (const long long*)a.hp, off, a.adj, vis, (uint32_t*)nullptr,
                       a.P, q[nxt], &sc->qcount[nxt]);
    CC_LAUNCH_CHECK();
    cur = nxt;
    ++a.sample_rounds;
  }
  // After the last wake every vertex is visited; the last expansion claimed
  // nothing new.  Relabel each cluster to its minimum member.
  hipLaunchKernelGGL(k_min_member, dim3(grid_for(n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, n, (const int32_t*)a.P,
                     mn);
  hipLaunchKernelGGL(k_relabel, dim3(grid_for(n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, n, a.P,
                     (const int32_t*)mn);
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
