// Round-based finishes: Shiloach-Vishkin and the root-based Liu-Tarjan
// variants (ConnectIt Section 3.3 "Other Min-Based Algorithms", appendix
// "Shiloach-Vishkin" and "Liu-Tarjan Algorithms").
//
// Both keep the parent array min-based (a parent only ever decreases, so
// P[x] <= x holds throughout), work over the edges of the candidate vertices
// (the most frequent sampled component is skipped), and stop after the first
// round that changes nothing.
#include "cc_frontier.h"
#include "cc_static.h"

namespace cc {

constexpr int kRoundCap = 100000;

// ---- Shiloach-Vishkin ------------------------------------------------------
// Hook: for an edge (u, v) with labels l < h, if h was a root at the start of
// the round, writeMin(P[h], l).  Then FullShortcut: every vertex points at its
// root, and the snapshot of roots is refreshed.
struct SvHook {
  int32_t* P;
  const int32_t* prev;
  __device__ __forceinline__ bool operator()(int32_t u, int32_t v, int64_t) const {
    const int32_t pu = ld(P + u), pv = ld(P + v);
    if (pu == pv) return false;
    const int32_t l = pu < pv ? pu : pv;
    const int32_t h = pu < pv ? pv : pu;
    if (prev[h] != h) return false;
    // P[h] only decreases: skip the atomic when another edge already did better
    if (ld(P + h) > l) amin(P + h, l);
    return true;
  }
};

// Pointer-jumps every vertex to its root; optionally writes the snapshot and
// raises `flag` when a parent changed.
__global__ void k_full_shortcut(int64_t n, int32_t* P, int32_t* snap, uint32_t* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool any = false;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    if (v < n) {
      const int32_t p = ld(P + v);
      int32_t r = p;
      if (p != (int32_t)v) {
        r = find_naive(P, p);
        if (r != p) {
          st(P + v, r);
          any = true;
        }
      }
      if (snap) snap[v] = r;
    }
  }
  if (flag) wave_flag(any, flag);
}

// One shortcut step: P[v] <- P[P[v]].
__global__ void k_shortcut_one(int64_t n, int32_t* P, uint32_t* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool any = false;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    if (v < n) {
      const int32_t p = ld(P + v);
      const int32_t pp = ld(P + p);
      if (pp != p) {
        amin(P + v, pp);
        any = true;
      }
    }
  }
  wave_flag(any, flag);
}

__global__ void k_copy_i32(int64_t n, const int32_t* __restrict__ src, int32_t* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

static cc_status read_flag(StaticArgs& a, uint32_t* out) {
  CC_HIP(hipMemcpyAsync(&a.ctx->host->changed, &a.ctx->dev->changed, 4, hipMemcpyDeviceToHost, a.s));
  CC_HIP(hipStreamSynchronize(a.s));
  *out = a.ctx->host->changed;
  return CC_OK;
}

template <typename I>
cc_status finish_sv(StaticArgs& a) {
  DevScalars* sc = a.ctx->dev;
  int32_t* prev = a.count;  // frequency counts are no longer needed
  const unsigned g = grid_for(a.n, kFBlock, 4096);
  // labels are fully compressed after sampling, so prev = P is a root snapshot
  hipLaunchKernelGGL(k_full_shortcut, dim3(g), dim3(kFBlock), 0, a.s, a.n, a.P, prev, (uint32_t*)nullptr);
  for (int round = 0;; ++round) {
    if (round >= kRoundCap) return fail(CC_ELIVELOCK, "Shiloach-Vishkin exceeded %d rounds", kRoundCap);
    if (a.ctx->round_limit > 0 && round >= a.ctx->round_limit)
      return fail(CC_ELIVELOCK, "Shiloach-Vishkin reached the context's round limit (%d)", a.ctx->round_limit);
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, a.s, &sc->changed, 0u);
    visit_candidates(a.s, a.lists(), (const I*)a.off, a.adj, SvHook{a.P, prev}, &sc->changed);
    hipLaunchKernelGGL(k_full_shortcut, dim3(g), dim3(kFBlock), 0, a.s, a.n, a.P, prev, (uint32_t*)nullptr);
    CC_LAUNCH_CHECK();
    ++a.finish_rounds;
    uint32_t changed = 0;
    cc_status st = read_flag(a, &changed);
    if (st != CC_OK) return st;
    if (!changed) break;
  }
  return CC_OK;
}

// ---- Liu-Tarjan (root-based) ------------------------------------------------
// update(x, c): with RootUp, only if x was a root when the round started
// (Q[x] == x); the parent becomes min(P[x], c).
__device__ __forceinline__ bool lt_update(int32_t* P, const int32_t* Q, int32_t x, int32_t c) {
  if (Q[x] != x) return false;
  if (c >= ld(P + x)) return false;
  return c < amin(P + x, c);
}

// Connect: the endpoints are each other's candidates.  ParentConnect: the
// endpoints' parents (from the round-start snapshot) are each other's
// candidates.
template <bool PARENT>
struct LtConnect {
  int32_t* P;
  const int32_t* Q;
  __device__ __forceinline__ bool operator()(int32_t v, int32_t w, int64_t) const {
    if (PARENT) {
      const int32_t pv = Q[v], pw = Q[w];
      if (pv == pw) return false;
      const bool x = lt_update(P, Q, pv, pw);
      const bool y = lt_update(P, Q, pw, pv);
      return x || y;
    }
    if (v == w) return false;
    const bool x = lt_update(P, Q, v, w);
    const bool y = lt_update(P, Q, w, v);
    return x || y;
  }
};

// Copies the candidates' edges into an explicit list (needed by Alter).
// The grid bin's edges take positions [0, hp[c3]) directly (their degree
// prefix exists); the other bins follow: a wave takes 64 candidates, scans
// their degrees and reserves the whole tile's range with one atomic.  A
// self-loop leaves a dead entry (eu = -1).
__global__ void k_lt_emit_base(const long long* hp, const DevScalars* sc, unsigned long long* cnt) {
  *cnt = (unsigned long long)hp[sc->bin_count[3]];
}

template <typename I>
__global__ void __launch_bounds__(kFBlock) k_lt_emit_heavy(const int32_t* __restrict__ heavy, const DevScalars* sc,
                                                           const long long* __restrict__ hp, const I* __restrict__ off,
                                                           const int32_t* __restrict__ adj, int32_t* eu, int32_t* ev) {
  const int64_t c = sc->bin_count[3];
  if (c == 0) return;
  const long long T = hp[c];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (long long base = blockIdx.x * (int64_t)blockDim.x; base < T; base += stride) {
    const long long e = base + threadIdx.x;
    const long long e0 = base + (threadIdx.x / kWave) * kWave;
    if (e < T) {
      const int64_t i = heavy_owner_tile(hp, c, e0, e);
      const int32_t u = heavy[i];
      const int32_t w = adj[(int64_t)off[u] + (e - hp[i])];
      eu[e] = u == w ? -1 : u;
      ev[e] = w;
    }
  }
}

template <typename I>
__global__ void __launch_bounds__(kFBlock) k_lt_emit(int64_t n, const int32_t* __restrict__ cand,
                                                     const int32_t* __restrict__ big, const DevScalars* sc,
                                                     const I* __restrict__ off, const int32_t* __restrict__ adj,
                                                     int32_t* eu, int32_t* ev, unsigned long long* cnt) {
  constexpr int W = kFBlock / kWave;
  __shared__ int32_t tpre[W][kWave + 1];
  __shared__ int64_t tbeg[W][kWave];
  __shared__ int32_t tu[W][kWave];
  const int wv = threadIdx.x / kWave, lane = lane_id();
  const int64_t c0 = sc->bin_count[0], c1 = sc->bin_count[1], c2 = sc->bin_count[2];
  const int64_t total_c = c0 + c1 + c2;
  const int64_t tiles = (total_c + kWave - 1) / kWave;
  const int64_t waves = (int64_t)gridDim.x * W;
  for (int64_t tile = blockIdx.x * (int64_t)W + wv; tile < tiles; tile += waves) {
    const int64_t i = tile * kWave + lane;
    int32_t u = 0;
    int64_t b = 0, d = 0;
    if (i < total_c) {
      u = i < c0 ? cand[i] : (i < c0 + c1 ? big[i - c0] : big[n - 1 - (i - c0 - c1)]);
      b = (int64_t)off[u];
      d = (int64_t)off[u + 1] - b;   // <= kThrGrid in these bins
    }
    int32_t inc = (int32_t)d;
    for (int o = 1; o < kWave; o <<= 1) {
      const int32_t y = __shfl_up(inc, o, kWave);
      if (lane >= o) inc += y;
    }
    const int32_t total = __shfl(inc, kWave - 1, kWave);
    tpre[wv][lane] = inc - (int32_t)d;
    tbeg[wv][lane] = b;
    tu[wv][lane] = u;
    unsigned long long base = 0;
    if (lane == 0 && total > 0)
      base = __hip_atomic_fetch_add(cnt, (unsigned long long)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    base = __shfl(base, 0, kWave);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int32_t e = lane; e < total; e += kWave) {
      int lo = 0, hi = kWave - 1;   // last row whose start <= e
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tpre[wv][mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      const int32_t uu = tu[wv][lo];
      const int32_t w = adj[tbeg[wv][lo] + (e - tpre[wv][lo])];
      eu[base + e] = uu == w ? -1 : uu;
      ev[base + e] = w;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <class Op>
__global__ void k_edge_list(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                            const unsigned long long* cnt, Op op, uint32_t* flag) {
  const int64_t c = (int64_t)*cnt;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool any = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += stride) {
    const int32_t a = eu[i];
    if (a < 0) continue;
    any |= op(a, ev[i], i);
  }
  wave_flag(any, flag);
}

// Alter: replace every live edge (v, w) by (P[v], P[w]); a self-loop dies.
__global__ void k_lt_alter(int32_t* eu, int32_t* ev, const unsigned long long* cnt, const int32_t* P,
                           uint32_t* flag) {
  const int64_t c = (int64_t)*cnt;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool any = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += stride) {
    const int32_t a = eu[i];
    if (a < 0) continue;
    const int32_t b = ev[i];
    const int32_t pa = ld(P + a), pb = ld(P + b);
    if (pa == pb) {
      eu[i] = -1;
    } else if (pa != a || pb != b) {
      eu[i] = pa;
      ev[i] = pb;
      any = true;
    }
  }
  wave_flag(any, flag);
}

template <typename I, bool PARENT>
static cc_status lt_rounds(StaticArgs& a) {
  DevScalars* sc = a.ctx->dev;
  const uint32_t rules = a.v->lt_rules;
  const bool full = rules & CC_LT_FULL_SHORTCUT;
  const bool alter = rules & CC_LT_ALTER;
  int32_t* Q = a.count;
  int32_t* eu = nullptr;
  int32_t* ev = nullptr;
  unsigned long long* ecnt = (unsigned long long*)&sc->frontier_edges;
  const unsigned g = grid_for(a.n, kFBlock, 4096);
  if (alter) {
    eu = (int32_t*)(a.ws + a.L.edges);
    ev = (int32_t*)(a.ws + a.L.edges + align256((size_t)a.m * 4));
    hipLaunchKernelGGL(k_lt_emit_base, dim3(1), dim3(1), 0, a.s, (const long long*)a.hp, (const DevScalars*)sc, ecnt);
    hipLaunchKernelGGL(k_lt_emit_heavy<I>, dim3(2048), dim3(kFBlock), 0, a.s, (const int32_t*)a.heavy,
                       (const DevScalars*)sc, (const long long*)a.hp, (const I*)a.off, a.adj, eu, ev);
    hipLaunchKernelGGL(k_lt_emit<I>, dim3(grid_for(a.n, kFBlock, 2048)), dim3(kFBlock), 0, a.s, a.n,
                       (const int32_t*)a.cand, (const int32_t*)a.big, (const DevScalars*)sc, (const I*)a.off, a.adj,
                       eu, ev, ecnt);
  }
  for (int round = 0;; ++round) {
    if (round >= kRoundCap) return fail(CC_ELIVELOCK, "Liu-Tarjan exceeded %d rounds", kRoundCap);
    if (a.ctx->round_limit > 0 && round >= a.ctx->round_limit)
      return fail(CC_ELIVELOCK, "Liu-Tarjan reached the context's round limit (%d)", a.ctx->round_limit);
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, a.s, &sc->changed, 0u);
    hipLaunchKernelGGL(k_copy_i32, dim3(g), dim3(kFBlock), 0, a.s, a.n, (const int32_t*)a.P, Q);
    LtConnect<PARENT> op{a.P, Q};
    if (alter) {
      hipLaunchKernelGGL(k_edge_list<LtConnect<PARENT>>, dim3(grid_for(a.m, kFBlock, 8192)), dim3(kFBlock), 0, a.s,
                         (const int32_t*)eu, (const int32_t*)ev, (const unsigned long long*)ecnt, op, &sc->changed);
    } else {
      visit_candidates(a.s, a.lists(), (const I*)a.off, a.adj, op, &sc->changed);
    }
    if (full) hipLaunchKernelGGL(k_full_shortcut, dim3(g), dim3(kFBlock), 0, a.s, a.n, a.P, (int32_t*)nullptr,
                                 &sc->changed);
    else hipLaunchKernelGGL(k_shortcut_one, dim3(g), dim3(kFBlock), 0, a.s, a.n, a.P, &sc->changed);
    if (alter)
      hipLaunchKernelGGL(k_lt_alter, dim3(grid_for(a.m, kFBlock, 8192)), dim3(kFBlock), 0, a.s, eu, ev,
                         (const unsigned long long*)ecnt, (const int32_t*)a.P, &sc->changed);
    CC_LAUNCH_CHECK();
    ++a.finish_rounds;
    uint32_t changed = 0;
    cc_status st = read_flag(a, &changed);
    if (st != CC_OK) return st;
    if (!changed) break;
  }
  return CC_OK;
}

// Rounds of SV or a root-based LT variant over an explicit edge list
// (eu[i] < 0: dead entry; *ecnt entries on the device, at most cap): the
// batch-insert step of a stream whose finish is SV or LT (the paper's
// type-2 streaming algorithms, which must process insertions in batches).
// P is the stream's min-based forest; Q is n int32 of scratch for the
// round snapshot.  Alter rewrites eu/ev.  Synchronises s once per round.
cc_status edge_list_rounds(cc_ctx* ctx, hipStream_t s, const cc_variant& v, int64_t n, int32_t* P, int32_t* Q,
                           int32_t* eu, int32_t* ev, const unsigned long long* ecnt, int64_t cap, int32_t* rounds) {
  DevScalars* sc = ctx->dev;
  const unsigned g = grid_for(n, kFBlock, 4096);
  const unsigned ge = grid_for(cap, kFBlock, 8192);
  const bool sv = v.finish == CC_FIN_SV;
  const bool parent = (v.lt_rules & 3u) == CC_LT_PARENT_CONNECT;
  const bool full = v.lt_rules & CC_LT_FULL_SHORTCUT;
  const bool alter = v.lt_rules & CC_LT_ALTER;
  *rounds = 0;
  // SV hooks only roots of the round-start snapshot: start from a flat forest
  if (sv) hipLaunchKernelGGL(k_full_shortcut, dim3(g), dim3(kFBlock), 0, s, n, P, Q, (uint32_t*)nullptr);
  for (int round = 0;; ++round) {
    if (round >= kRoundCap) return fail(CC_ELIVELOCK, "batch rounds exceeded %d", kRoundCap);
    if (ctx->round_limit > 0 && round >= ctx->round_limit)
      return fail(CC_ELIVELOCK, "batch rounds reached the context's round limit (%d)", ctx->round_limit);
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, &sc->changed, 0u);
    if (sv) {
      hipLaunchKernelGGL(k_edge_list<SvHook>, dim3(ge), dim3(kFBlock), 0, s, (const int32_t*)eu, (const int32_t*)ev,
                         ecnt, SvHook{P, Q}, &sc->changed);
      hipLaunchKernelGGL(k_full_shortcut, dim3(g), dim3(kFBlock), 0, s, n, P, Q, (uint32_t*)nullptr);
    } else {
      hipLaunchKernelGGL(k_copy_i32, dim3(g), dim3(kFBlock), 0, s, n, (const int32_t*)P, Q);
      if (parent)
        hipLaunchKernelGGL(k_edge_list<LtConnect<true>>, dim3(ge), dim3(kFBlock), 0, s, (const int32_t*)eu,
                           (const int32_t*)ev, ecnt, LtConnect<true>{P, Q}, &sc->changed);
      else
        hipLaunchKernelGGL(k_edge_list<LtConnect<false>>, dim3(ge), dim3(kFBlock), 0, s, (const int32_t*)eu,
                           (const int32_t*)ev, ecnt, LtConnect<false>{P, Q}, &sc->changed);
      if (full) hipLaunchKernelGGL(k_full_shortcut, dim3(g), dim3(kFBlock), 0, s, n, P, (int32_t*)nullptr, &sc->changed);
      else hipLaunchKernelGGL(k_shortcut_one, dim3(g), dim3(kFBlock), 0, s, n, P, &sc->changed);
      if (alter)
        hipLaunchKernelGGL(k_lt_alter, dim3(ge), dim3(kFBlock), 0, s, eu, ev, ecnt, (const int32_t*)P, &sc->changed);
    }
    CC_LAUNCH_CHECK();
    ++*rounds;
    CC_HIP(hipMemcpyAsync(&ctx->host->changed, &sc->changed, 4, hipMemcpyDeviceToHost, s));
    CC_HIP(hipStreamSynchronize(s));
    if (!ctx->host->changed) break;
  }
  return CC_OK;
}

// ---- label propagation (appendix "Label Propagation") ---------------------
// Labels are the parent array read as labels.  The frequent sampled class
// is first relabelled to -1, below every id, so its vertices never change
// and their label spreads to every vertex connected to them (the paper's
// way of composing label propagation with sampling).  Rounds follow the
// appendix's frontier: round 0 applies every candidate edge both ways with
// writeMin (the frontier is every vertex); afterwards a round visits only
// the edges of the vertices whose label dropped in the round before.  The
// lane whose writeMin lowers a label sets that vertex's bit in a bitmap; the
// next round's frontier is built from the bitmap (bits cleared as they are
// read) into the same four degree bins as the candidate lists, so the same
// edge visitors balance its rows.  Rounds stop when no bit was set.  Then
// the -1 class takes its smallest member as its label; every other class
// already carries its minimum (the sampled labels are class minima), so the
// result is the canonical labelling and a star forest.
//
// One change of schedule against the appendix: a lane that walks a row of
// the thread bin and lowers the label of a neighbour whose own row is also
// short pushes that neighbour onto a small stack in LDS and walks its row
// next (depth first, at most kLpChase rows per frontier vertex), instead of
// leaving it to the next round; only what does not fit gets a bit.  With
// rounds alone a label moves one edge per round, and on a graph whose ids
// follow its geometry (a lattice) every vertex then takes a new, slightly
// smaller label in almost every round, so the work grows with n times the
// diameter.  The fixed point is the same: every vertex whose label drops
// has its row walked afterwards, with a label read after the drop, either
// by the lane that lowered it or in the next round.
struct LpOp {
  int32_t* P;
  uint32_t* chg;  // bit per vertex: its label dropped and its row is still to walk
  __device__ __forceinline__ bool operator()(int32_t u, int32_t w, int64_t) const {
    const int32_t a = ld(P + u), c = ld(P + w);
    if (a < c) {
      if (amin(P + w, a) <= a) return false;
      bit_claim(chg, w);
      return true;
    }
    if (c < a) {
      if (amin(P + u, c) <= c) return false;
      bit_claim(chg, u);
      return true;
    }
    return false;
  }
};

constexpr int kLpStack = 16;  // rows a lane keeps waiting in LDS
constexpr int kLpChase = 64;  // rows a lane walks per frontier vertex beyond its own

// Thread-bin part of a label propagation round: one lane per frontier
// vertex, with the depth-first push described above.
template <typename I>
__device__ __forceinline__ void lp_thread_part(int64_t bid, int64_t nb, const int32_t* __restrict__ list,
                                               const int32_t* bins, const I* __restrict__ off,
                                               const int32_t* __restrict__ adj, int32_t* P, uint32_t* chg,
                                               int32_t (*stk)[kFBlock], uint32_t* flag) {
  const int64_t cnt = bins[0];
  const int t = threadIdx.x;
  const int64_t stride = nb * blockDim.x;
  bool any = false;
  for (int64_t i = bid * (int64_t)blockDim.x + t; i < cnt; i += stride) {
    int32_t x = list[i];
    int sp = 0, budget = kLpChase;
    for (;;) {
      int32_t a = ld(P + x);
      const int64_t e = (int64_t)off[x + 1];
      for (int64_t j = (int64_t)off[x]; j < e; ++j) {
        const int32_t w = adj[j];
        const int32_t c = ld(P + w);
        if (a < c) {
          if (amin(P + w, a) > a) {
            bool walk = false;
            if (sp < kLpStack && budget > 0) walk = (int64_t)off[w + 1] - (int64_t)off[w] <= kThrWave;
            if (walk) {
              stk[sp++][t] = w;
              --budget;
            } else {
              bit_claim(chg, w);
              any = true;
            }
          }
        } else if (c < a) {
          const int32_t old = amin(P + x, c);
          if (old > c) {
            // the entries before j got the larger label: walk the row again
            bit_claim(chg, x);
            any = true;
          }
          a = old < c ? old : c;
        }
      }
      if (sp == 0) break;
      x = stk[--sp][t];
    }
  }
  if (flag) wave_flag(any, flag);
}

// One label propagation round over degree-binned lists (the candidates in
// round 0, a frontier afterwards); the block layout of k_visit_all.
template <typename I>
__global__ void __launch_bounds__(kFBlock) k_lp_visit(int64_t n, int64_t g0, int64_t g1, int64_t g2,
                                                      const int32_t* __restrict__ cand,
                                                      const int32_t* __restrict__ big,
                                                      const int32_t* __restrict__ heavy,
                                                      const long long* __restrict__ hp, const int32_t* bins,
                                                      const I* __restrict__ off, const int32_t* __restrict__ adj,
                                                      int32_t* P, uint32_t* chg, uint32_t* flag) {
  __shared__ int32_t stk[kLpStack][kFBlock];
  int64_t b = blockIdx.x;
  if (b < g0) return lp_thread_part<I>(b, g0, cand, bins, off, adj, P, chg, stk, flag);
  b -= g0;
  const LpOp op{P, chg};
  if (b < g1) return visit_wave_part<LpOp, I>(b, g1, big, bins, off, adj, op, flag);
  b -= g1;
  if (b < g2) return visit_block_part<LpOp, I>(b, g2, n, big, bins, off, adj, op, flag);
  b -= g2;
  visit_heavy_part<LpOp, I>(b, (int64_t)gridDim.x - g0 - g1 - g2, heavy, &bins[3], hp, off, adj, op, flag);
}

template <typename I>
static void lp_round(hipStream_t s, const CandLists& L, const I* off, const int32_t* adj, int32_t* P, uint32_t* chg,
                     uint32_t* flag) {
  int64_t g[4];
  visit_grids(L.n, g);
  hipLaunchKernelGGL(k_lp_visit<I>, dim3((unsigned)(g[0] + g[1] + g[2] + g[3])), dim3(kFBlock), 0, s, L.n, g[0],
                     g[1], g[2], L.cand, L.big, L.heavy, L.hp, L.bins, off, adj, P, chg, flag);
}

// Next frontier from the change bitmap: every set bit is cleared and its
// vertex appended to the bin of its degree (thread bin to q0, wave bin to
// the front of q1, block bin to the back of q1, grid bin to `heavy`), with
// one counter add per wave and bin.  Also zeroes the other round's bin
// counters and the change flag for the visit that follows.
template <typename I>
__global__ void __launch_bounds__(kFBlock) k_lp_frontier(int64_t n, uint32_t* __restrict__ chg,
                                                         const I* __restrict__ off, int32_t* __restrict__ q0,
                                                         int32_t* __restrict__ q1, int32_t* __restrict__ heavy,
                                                         int32_t* bins, int32_t* other_bins, uint32_t* changed) {
  if (blockIdx.x == 0 && threadIdx.x < 4) other_bins[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) *changed = 0u;
  const int64_t words = (n + 31) >> 5;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += stride) {
    uint32_t w = chg[i];
    if (w) chg[i] = 0u;
    while (__ballot(w != 0u)) {
      const bool has = w != 0u;
      int64_t v = 0, deg = 0;
      if (has) {
        v = (i << 5) + (__ffs((int)w) - 1);
        w &= w - 1u;
        deg = (int64_t)off[v + 1] - (int64_t)off[v];
      }
      const int bin = !has ? -1 : deg <= kThrWave ? 0 : deg <= kThrBlock ? 1 : deg <= kThrGrid ? 2 : 3;
      wave_append(bin == 0, (int32_t)v, q0, (uint32_t*)&bins[0]);
      wave_append(bin == 1, (int32_t)v, q1, (uint32_t*)&bins[1]);
      wave_append(bin == 3, (int32_t)v, heavy, (uint32_t*)&bins[3]);
      const uint64_t mb = __ballot(bin == 2);
      if (mb) {
        const int leader = __ffsll((unsigned long long)mb) - 1;
        uint32_t base = 0;
        if (lane_id() == leader)
          base = __hip_atomic_fetch_add((uint32_t*)&bins[2], (uint32_t)__popcll(mb), __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
        base = __shfl(base, leader, kWave);
        if (bin == 2) q1[n - 1 - (int64_t)(base + (uint32_t)__popcll(mb & lanemask_lt()))] = (int32_t)v;
      }
    }
  }
}

__global__ void k_lp_begin(int32_t* bins1, uint32_t* changed) {
  if (threadIdx.x < 4) bins1[threadIdx.x] = 0;
  if (threadIdx.x == 0) *changed = 0u;
}

__global__ void k_lp_mark(int64_t n, int32_t* P, const DevScalars* sc) {
  const int32_t L = sc->lmax;
  if (L < 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride)
    if (P[v] == L) P[v] = -1;
}

// Per-block minimum vertex id labelled -1 (n when none).
__global__ void __launch_bounds__(kFBlock) k_lp_min(int64_t n, const int32_t* __restrict__ P,
                                                    int32_t* __restrict__ part) {
  __shared__ int32_t red[kFBlock / kWave];
  int32_t m = (int32_t)(n < 0x7fffffff ? n : 0x7fffffff);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride)
    if (P[v] == -1 && (int32_t)v < m) m = (int32_t)v;
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t y = __shfl_xor(m, o, kWave);
    m = y < m ? y : m;
  }
  if (lane_id() == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kFBlock / kWave; ++i) m = red[i] < m ? red[i] : m;
    part[blockIdx.x] = m;
  }
}

__global__ void k_lp_fix(int64_t n, int32_t* P, const int32_t* __restrict__ part, int nparts) {
  __shared__ int32_t s_min;
  if (threadIdx.x == 0) {
    int32_t m = 0x7fffffff;
    for (int i = 0; i < nparts; ++i) m = part[i] < m ? part[i] : m;
    s_min = m;
  }
  __syncthreads();
  const int32_t m = s_min;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride)
    if (P[v] == -1) P[v] = m;
}

template <typename I>
cc_status finish_lp(StaticArgs& a) {
  DevScalars* sc = a.ctx->dev;
  const int64_t n = a.n;
  const unsigned g = grid_for(n, kFBlock, 4096);
  // frontier state: the change bitmap, the thread bin and the wave/block
  // bins in the frontier queues (free after sampling), the grid bin in the
  // candidates' heavy list (free once round 0 has visited it)
  uint32_t* chg = (uint32_t*)(a.ws + a.L.bits);
  int32_t* q0 = (int32_t*)(a.ws + a.L.queue);
  int32_t* q1 = (int32_t*)(a.ws + a.L.queue + align256((size_t)n * 4));
  const int64_t words = (n + 31) >> 5;
  // whether any candidate row is long enough for the grid bin (then each
  // frontier needs that bin's degree prefix)
  CC_HIP(hipMemcpyAsync(a.ctx->host->bin_count, sc->bin_count, sizeof(sc->bin_count), hipMemcpyDeviceToHost, a.s));
  CC_HIP(hipStreamSynchronize(a.s));
  const bool grid_bin = a.ctx->host->bin_count[3] > 0;
  hipLaunchKernelGGL(k_lp_mark, dim3(g), dim3(kFBlock), 0, a.s, n, a.P, (const DevScalars*)sc);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(words, kFBlock, 4096)), dim3(kFBlock), 0, a.s, chg, words, 0u);
  hipLaunchKernelGGL(k_lp_begin, dim3(1), dim3(64), 0, a.s, sc->fbin[1], &sc->changed);
  const unsigned gf = grid_for(words, kFBlock, 2048);
  for (int round = 0;; ++round) {
    if (round >= kRoundCap) return fail(CC_ELIVELOCK, "label propagation exceeded %d rounds", kRoundCap);
    if (a.ctx->round_limit > 0 && round >= a.ctx->round_limit)
      return fail(CC_ELIVELOCK, "label propagation reached the context's round limit (%d)", a.ctx->round_limit);
    if (round == 0) {
      lp_round<I>(a.s, a.lists(), (const I*)a.off, a.adj, a.P, chg, &sc->changed);
    } else {
      int32_t* bins = sc->fbin[round & 1];
      hipLaunchKernelGGL(k_lp_frontier<I>, dim3(gf), dim3(kFBlock), 0, a.s, n, chg, (const I*)a.off, q0, q1,
                         a.heavy, bins, sc->fbin[(round + 1) & 1], &sc->changed);
      if (grid_bin) heavy_prefix<I>(a.s, a.heavy, &bins[3], a.hcap, (const I*)a.off, a.tsum, a.hp);
      const CandLists fl{n, q0, q1, a.heavy, a.hp, bins};
      lp_round<I>(a.s, fl, (const I*)a.off, a.adj, a.P, chg, &sc->changed);
    }
    CC_LAUNCH_CHECK();
    ++a.finish_rounds;
    uint32_t changed = 0;
    cc_status st = read_flag(a, &changed);
    if (st != CC_OK) return st;
    if (!changed) break;
  }
  // per-block minima in the count array (free after the compaction)
  const unsigned gm = grid_for(n, kFBlock, 1024);
  hipLaunchKernelGGL(k_lp_min, dim3(gm), dim3(kFBlock), 0, a.s, n, (const int32_t*)a.P, a.count);
  hipLaunchKernelGGL(k_lp_fix, dim3(g), dim3(kFBlock), 0, a.s, n, a.P, (const int32_t*)a.count, (int)gm);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

// ---- Liu-Tarjan, non-root-based variants ------------------------------------
// Any vertex may take a smaller candidate as its parent, so a non-root can
// move between trees and the method is not monotone; it is composed with
// sampling as label propagation is (appendix "Correctness for Other
// Min-Based Methods"): the frequent sampled class is relabelled to a
// virtual vertex -1, below every id, which never changes and whose own
// parent is itself.  Edges in the Alter list may then have -1 as an
// endpoint, so a dead entry is marked with kDead instead.
constexpr int32_t kDead = (int32_t)0x80000000;

__device__ __forceinline__ int32_t vsnap(const int32_t* Q, int32_t x) { return x < 0 ? -1 : Q[x]; }

// update(x, c) without RootUp: the parent of any real vertex becomes
// min(P[x], c).
__device__ __forceinline__ bool lt_update_any(int32_t* P, int32_t x, int32_t c) {
  if (x < 0) return false;
  if (c >= ld(P + x)) return false;
  return c < amin(P + x, c);
}

// CONN 0 Connect (the endpoints are each other's candidates), 1
// ParentConnect (the endpoints' round-start parents, for those parents),
// 2 ExtendedConnect (the round-start parents, for both the endpoints and
// their parents).
template <int CONN>
struct LtConnectAny {
  int32_t* P;
  const int32_t* Q;
  __device__ __forceinline__ bool operator()(int32_t v, int32_t w, int64_t) const {
    if (CONN == 0) {
      if (v == w) return false;
      const bool x = lt_update_any(P, v, w);
      const bool y = lt_update_any(P, w, v);
      return x || y;
    }
    const int32_t pv = vsnap(Q, v), pw = vsnap(Q, w);
    if (pv == pw) return false;
    bool ch = lt_update_any(P, pv, pw);
    ch |= lt_update_any(P, pw, pv);
    if (CONN == 2) {
      ch |= lt_update_any(P, v, pw);
      ch |= lt_update_any(P, w, pv);
    }
    return ch;
  }
};

template <class Op>
__global__ void k_edge_list_v(const int32_t* __restrict__ eu, const int32_t* __restrict__ ev,
                              const unsigned long long* cnt, Op op, uint32_t* flag) {
  const int64_t c = (int64_t)*cnt;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool any = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += stride) {
    const int32_t a = eu[i];
    if (a == kDead) continue;
    any |= op(a, ev[i], i);
  }
  wave_flag(any, flag);
}

// Emitted self-loops (-1) become kDead before -1 means the virtual vertex.
__global__ void k_mark_dead(int32_t* eu, const unsigned long long* cnt) {
  const int64_t c = (int64_t)*cnt;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += stride)
    if (eu[i] == -1) eu[i] = kDead;
}

__global__ void k_lt_alter_v(int32_t* eu, int32_t* ev, const unsigned long long* cnt, const int32_t* P,
                             uint32_t* flag) {
  const int64_t c = (int64_t)*cnt;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool any = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += stride) {
    const int32_t a = eu[i];
    if (a == kDead) continue;
    const int32_t b = ev[i];
    const int32_t pa = a < 0 ? -1 : ld(P + a), pb = b < 0 ? -1 : ld(P + b);
    if (pa == pb) {
      eu[i] = kDead;
    } else if (pa != a || pb != b) {
      eu[i] = pa;
      ev[i] = pb;
      any = true;
    }
  }
  wave_flag(any, flag);
}

// Shortcut with the virtual vertex: one step P[v] = P[P[v]], or the full
// walk to the root (a real root or -1).  Parents only decrease.
__global__ void k_shortcut_v(int64_t n, int32_t* P, int full, uint32_t* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool any = false;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t p = ld(P + v);
    if (p < 0 || p == (int32_t)v) continue;
    int32_t r = ld(P + p);
    if (full) {
      int32_t q = p;
      while (r >= 0 && r != q) {
        q = r;
        r = ld(P + q);
      }
      if (r >= 0) r = q;  // a real root; else the walk ended at -1
    }
    if (r < p) {
      amin(P + v, r);
      any = true;
    }
  }
  wave_flag(any, flag);
}

template <typename I, int CONN>
static cc_status lt_rounds_nonroot(StaticArgs& a) {
  DevScalars* sc = a.ctx->dev;
  const uint32_t rules = a.v->lt_rules;
  const bool full = rules & CC_LT_FULL_SHORTCUT;
  const bool alter = rules & CC_LT_ALTER;
  int32_t* Q = a.count;
  int32_t* eu = nullptr;
  int32_t* ev = nullptr;
  unsigned long long* ecnt = (unsigned long long*)&sc->frontier_edges;
  const unsigned g = grid_for(a.n, kFBlock, 4096);
  hipLaunchKernelGGL(k_lp_mark, dim3(g), dim3(kFBlock), 0, a.s, a.n, a.P, (const DevScalars*)sc);
  if (alter) {
    eu = (int32_t*)(a.ws + a.L.edges);
    ev = (int32_t*)(a.ws + a.L.edges + align256((size_t)a.m * 4));
    hipLaunchKernelGGL(k_lt_emit_base, dim3(1), dim3(1), 0, a.s, (const long long*)a.hp, (const DevScalars*)sc, ecnt);
    hipLaunchKernelGGL(k_lt_emit_heavy<I>, dim3(2048), dim3(kFBlock), 0, a.s, (const int32_t*)a.heavy,
                       (const DevScalars*)sc, (const long long*)a.hp, (const I*)a.off, a.adj, eu, ev);
    hipLaunchKernelGGL(k_lt_emit<I>, dim3(grid_for(a.n, kFBlock, 2048)), dim3(kFBlock), 0, a.s, a.n,
                       (const int32_t*)a.cand, (const int32_t*)a.big, (const DevScalars*)sc, (const I*)a.off, a.adj,
                       eu, ev, ecnt);
    hipLaunchKernelGGL(k_mark_dead, dim3(grid_for(a.m, kFBlock, 8192)), dim3(kFBlock), 0, a.s, eu,
                       (const unsigned long long*)ecnt);
  }
  for (int round = 0;; ++round) {
    if (round >= kRoundCap) return fail(CC_ELIVELOCK, "Liu-Tarjan exceeded %d rounds", kRoundCap);
    if (a.ctx->round_limit > 0 && round >= a.ctx->round_limit)
      return fail(CC_ELIVELOCK, "Liu-Tarjan reached the context's round limit (%d)", a.ctx->round_limit);
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, a.s, &sc->changed, 0u);
    hipLaunchKernelGGL(k_copy_i32, dim3(g), dim3(kFBlock), 0, a.s, a.n, (const int32_t*)a.P, Q);
    const LtConnectAny<CONN> op{a.P, Q};
    if (alter)
      hipLaunchKernelGGL(k_edge_list_v<LtConnectAny<CONN>>, dim3(grid_for(a.m, kFBlock, 8192)), dim3(kFBlock), 0,
                         a.s, (const int32_t*)eu, (const int32_t*)ev, (const unsigned long long*)ecnt, op,
                         &sc->changed);
    else
      visit_candidates(a.s, a.lists(), (const I*)a.off, a.adj, op, &sc->changed);
    hipLaunchKernelGGL(k_shortcut_v, dim3(g), dim3(kFBlock), 0, a.s, a.n, a.P, full ? 1 : 0, &sc->changed);
    if (alter)
      hipLaunchKernelGGL(k_lt_alter_v, dim3(grid_for(a.m, kFBlock, 8192)), dim3(kFBlock), 0, a.s, eu, ev,
                         (const unsigned long long*)ecnt, (const int32_t*)a.P, &sc->changed);
    CC_LAUNCH_CHECK();
    ++a.finish_rounds;
    uint32_t changed = 0;
    cc_status st = read_flag(a, &changed);
    if (st != CC_OK) return st;
    if (!changed) break;
  }
  // the virtual vertex's class takes its smallest member (minima of the
  // count array's blocks first; the snapshot is no longer needed)
  const unsigned gm = grid_for(a.n, kFBlock, 1024);
  hipLaunchKernelGGL(k_lp_min, dim3(gm), dim3(kFBlock), 0, a.s, a.n, (const int32_t*)a.P, a.count);
  hipLaunchKernelGGL(k_lp_fix, dim3(g), dim3(kFBlock), 0, a.s, a.n, a.P, (const int32_t*)a.count, (int)gm);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

template <typename I>
cc_status finish_lt(StaticArgs& a) {
  const uint32_t conn = a.v->lt_rules & 3u;
  if (!(a.v->lt_rules & CC_LT_ROOTUP)) {
    if (conn == CC_LT_PARENT_CONNECT) return lt_rounds_nonroot<I, 1>(a);
    if (conn == CC_LT_EXTENDED_CONNECT) return lt_rounds_nonroot<I, 2>(a);
    return lt_rounds_nonroot<I, 0>(a);
  }
  if (conn == CC_LT_PARENT_CONNECT) return lt_rounds<I, true>(a);
  return lt_rounds<I, false>(a);
}

template cc_status finish_sv<int32_t>(StaticArgs&);
template cc_status finish_sv<int64_t>(StaticArgs&);
template cc_status finish_lt<int32_t>(StaticArgs&);
template cc_status finish_lt<int64_t>(StaticArgs&);
template cc_status finish_lp<int32_t>(StaticArgs&);
template cc_status finish_lp<int64_t>(StaticArgs&);

}  // namespace cc
