// Static connectivity (ConnectIt Algorithm 1) on gfx950.
//
//   init            P[v] = v, frequency counters cleared          (Alg. 1 init)
//   sample          k-out: first edge + k-1 seeded picks, united with
//                   UF-Rem-CAS/SplitAtomicOne (Section 3.2 "k-out Sampling");
//                   BFS / LDD live in cc_sample.hip
//   compress_count  P[v] = root(v) (full compression) fused with the label
//                   histogram of IdentifyFrequent
//   frequent        L_max = most frequent label, ties to the smaller label
//   compact         candidates = {v : P[v] != L_max, deg(v) > 0}, binned by
//                   degree (thread / wave / block per vertex)
//   finish          union-find over every candidate's edges (appendix
//                   "Union Find Algorithms" meta-algorithm); SV / LT live in
//                   cc_rounds.hip
//   output          P[v] = root(v); count roots
//
// P is the caller's labels_out buffer: the parent array lives there for the
// whole call, so the final compression writes the answer in place.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "cc_device.h"
#include "cc_frontier.h"
#include "cc_internal.h"
#include "cc_static.h"

namespace cc {

// ---------------------------------------------------------------------------
// errors
static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

cc_status fail(cc_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

// ---------------------------------------------------------------------------
// phase timing
static hipEvent_t get_event(cc_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

PhaseScope::PhaseScope(cc_ctx* c, hipStream_t st, const char* nm) : ctx(c), s(st), name(nm) {
  // each recorded event makes the stream wait for the work before it, so a
  // measurement of one phase records only that phase's pair
  if (ctx && ctx->timing && (ctx->timing_only.empty() || ctx->timing_only == nm)) {
    a = get_event(ctx);
    if (a) (void)hipEventRecord(a, s);
  }
}

PhaseScope::~PhaseScope() {
  if (!a) return;
  hipEvent_t b = get_event(ctx);
  if (!b) return;
  (void)hipEventRecord(b, s);
  ctx->pending.push_back({name, a, b});
}

static void harvest(cc_ctx* ctx) {
  for (auto& r : ctx->pending) {
    (void)hipEventSynchronize(r.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    size_t i = 0;
    for (; i < ctx->phase_names.size(); ++i)
      if (ctx->phase_names[i] == r.name) break;
    if (i == ctx->phase_names.size()) {
      ctx->phase_names.push_back(r.name);
      ctx->phase_ms.push_back(0.0);
      ctx->phase_cnt.push_back(0);
    }
    ctx->phase_ms[i] += ms;
    ctx->phase_cnt[i] += 1;
    ctx->event_pool.push_back(r.a);
    ctx->event_pool.push_back(r.b);
  }
  ctx->pending.clear();
}

// ---------------------------------------------------------------------------
// variant rules
cc_status check_variant(const cc_variant* v, bool for_stream) {
  if (!v) return fail(CC_EINVAL, "variant is NULL");
  if (v->sample < CC_SAMPLE_NONE || v->sample > CC_SAMPLE_LDD) return fail(CC_EINVAL, "bad sample %d", v->sample);
  if (v->sample == CC_SAMPLE_KOUT) {
    if (v->kout_k < 1 || v->kout_k > 64) return fail(CC_EINVAL, "kout_k must be in [1, 64]");
    if (v->kout_mode < CC_KOUT_HYBRID || v->kout_mode > CC_KOUT_MAXDEG) return fail(CC_EINVAL, "bad kout_mode");
  }
  if (v->sample == CC_SAMPLE_BFS && (v->bfs_tries < 1 || v->bfs_tries > 64))
    return fail(CC_EINVAL, "bfs_tries must be in [1, 64]");
  if (v->sample == CC_SAMPLE_LDD) {
    if (!(v->ldd_beta > 0.f && v->ldd_beta < 1.f)) return fail(CC_EINVAL, "ldd_beta must be in (0, 1)");
    if (v->ldd_permute != 0) return fail(CC_EUNSUPPORTED, "ldd_permute != 0 is not built");
  }
  switch (v->finish) {
    case CC_FIN_UF_REM_CAS:
      if (v->splice < CC_SPLICE_SPLIT_ONE || v->splice > CC_SPLICE_ATOMIC) return fail(CC_EINVAL, "bad splice");
      if (v->find == CC_FIND_COMPRESS)
        return fail(CC_EINVAL,
                    "FindCompress is not a compress option of UF-Rem-CAS (with SpliceAtomic it is the paper's "
                    "incorrect combination)");
      if (v->find < CC_FIND_NAIVE || v->find > CC_FIND_ATOMIC_HALVE) return fail(CC_EINVAL, "bad find");
      break;
    case CC_FIN_UF_ASYNC:
    case CC_FIN_UF_EARLY:
    case CC_FIN_UF_HOOKS:
      if (v->find < CC_FIND_NAIVE || v->find > CC_FIND_COMPRESS) return fail(CC_EINVAL, "bad find");
      break;
    case CC_FIN_LP:
      if (for_stream) return fail(CC_EUNSUPPORTED, "label propagation is not a streaming algorithm");
      break;
    case CC_FIN_SV:
      break;
    case CC_FIN_LT: {
      uint32_t r = v->lt_rules;
      const uint32_t root[] = {CC_LT_CRSA, CC_LT_PRSA, CC_LT_PRS, CC_LT_CRFA, CC_LT_PRFA, CC_LT_PRF};
      const uint32_t nonroot[] = {CC_LT_CUSA, CC_LT_PUSA, CC_LT_PUS, CC_LT_EUSA, CC_LT_EUS,
                                  CC_LT_CUFA, CC_LT_PUFA, CC_LT_PUF, CC_LT_EUFA, CC_LT_EUF};
      bool is_root = false, is_nonroot = false;
      for (uint32_t x : root) is_root |= (r == x);
      for (uint32_t x : nonroot) is_nonroot |= (r == x);
      if (!is_root && !is_nonroot)
        return fail(CC_EUNSUPPORTED, "rules=%u is not one of the 16 Liu-Tarjan variants of the appendix", r);
      if (for_stream && !is_root)
        return fail(CC_EUNSUPPORTED, "stream finishes use the root-based Liu-Tarjan variants only");
      break;
    }
    default:
      return fail(CC_EINVAL, "bad finish %d", v->finish);
  }
  return CC_OK;
}

constexpr int kSegMaxHost = 8448;

WsLayout ws_layout(int64_t n, int64_t m, const cc_variant* v) {
  WsLayout L;
  size_t off = 0;
  const size_t n4 = align256((size_t)n * 4);
  L.count = off, off += n4;
  L.cand = off, off += n4;
  L.big = off, off += n4;
  // frontier state for BFS / LDD sampling and the selector's BFS probe
  L.bits = off, off += 3 * align256((size_t)((n + 31) / 32) * 4);
  L.queue = off, off += 2 * n4;
  L.hist = off, off += align256(4096 * 4);
  L.mlp = off, off += 65536;   // selector: feature partials, label stats, one MLP row
  if (v->finish == CC_FIN_LT && (v->lt_rules & CC_LT_ALTER)) L.edges = off, off += 2 * align256((size_t)m * 4);
  L.seg = off, off += align256((size_t)kSegMaxHost * 16) + 2 * align256((size_t)kSegMaxHost * 8) +
                     align256((size_t)kSegMaxHost / 4 * 16) + 2 * align256((size_t)kSegMaxHost / 4 * 8);
  {
    const size_t hcap = heavy_cap(m);  // vertices with degree above the frontier threshold
    L.heavy = off, off += align256(hcap * 4) + align256((hcap + 1) * 8) + align256((hcap / kHpTile + 3) * 8);
  }
  L.total = off + 256;
  return L;
}

// ---------------------------------------------------------------------------
// kernels
constexpr int kBlock = 256;
constexpr int64_t kStreamGridCap = 4096;
constexpr int64_t kVertexGridCap = (int64_t)1 << 21;  // up to 2^29 vertices at one per thread

__device__ __forceinline__ int64_t div_up_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }
__device__ __forceinline__ uint64_t lanemask_lt_dev() {
  const int l = __lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}


// Per-call device scalars back to their starting values.
__device__ __forceinline__ void reset_scalars(DevScalars* sc, long long* ncomp_user) {
  sc->changed = 0;
  sc->lmax_key = 0ull;
  sc->lmax = -1;
  sc->bfs_min = 0x7fffffff;
  for (int b = 0; b < 4; ++b) sc->bin_count[b] = 0;
  sc->cand_edges = 0;
  sc->num_components = 0;
  sc->lmax_size = 0;
  sc->bu_rounds = 0;
  sc->qcount[0] = sc->qcount[1] = 0;
  sc->frontier_edges = 0;
  sc->reached = 0;
  sc->flag2 = 0;
  if (ncomp_user) *ncomp_user = 0;
}


// P[v] = v and count[v] = 0, four vertices per lane with 16-byte stores;
// the first thread also resets the call's device scalars.
// P[v] = v for v < np (np >= n: a call restricted to the first n vertices
// still gives every vertex of the array a valid parent) and count[v] = 0 for
// v < n.
__global__ void k_init(int64_t n, int64_t np, int32_t* __restrict__ P, int32_t* __restrict__ count, int aligned,
                       DevScalars* sc, long long* ncomp_user) {
  if (blockIdx.x == 0 && threadIdx.x == 0) reset_scalars(sc, ncomp_user);
  const int64_t groups = div_up_dev(np, 4);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < groups; g += stride) {
    const int64_t v0 = 4 * g;
    if (aligned && v0 + 3 < np) {
      *(int4*)(P + v0) = make_int4((int)v0, (int)v0 + 1, (int)v0 + 2, (int)v0 + 3);
    } else {
      for (int j = 0; j < 4; ++j)
        if (v0 + j < np) P[v0 + j] = (int32_t)(v0 + j);
    }
    if (count && v0 < n) {
      if (aligned && v0 + 3 < n) {
        *(int4*)(count + v0) = make_int4(0, 0, 0, 0);
      } else {
        for (int j = 0; j < 4; ++j)
          if (v0 + j < n) count[v0 + j] = 0;
      }
    }
  }
}

// Loads off[v0 .. v0+4] (five entries) as int64.
__device__ __forceinline__ void load_off5(const int32_t* off, int64_t v0, bool vec, int64_t n, int64_t o[5]) {
  if (vec) {
    const int4 a = *(const int4*)(off + v0);
    o[0] = a.x, o[1] = a.y, o[2] = a.z, o[3] = a.w;
    o[4] = off[v0 + 4];
  } else {
    for (int j = 0; j < 5; ++j) o[j] = (v0 + j <= n) ? (int64_t)off[v0 + j] : 0;
  }
}
__device__ __forceinline__ void load_off5(const int64_t* off, int64_t v0, bool vec, int64_t n, int64_t o[5]) {
  if (vec) {
    const longlong2 a = *(const longlong2*)(off + v0);
    const longlong2 b = *(const longlong2*)(off + v0 + 2);
    o[0] = a.x, o[1] = a.y, o[2] = b.x, o[3] = b.y;
    o[4] = off[v0 + 4];
  } else {
    for (int j = 0; j < 5; ++j) o[j] = (v0 + j <= n) ? (int64_t)off[v0 + j] : 0;
  }
}
__device__ __forceinline__ void load4(const int32_t* p, int64_t v0, bool vec, int64_t n, int32_t x[4]) {
  if (vec) {
    const int4 a = *(const int4*)(p + v0);
    x[0] = a.x, x[1] = a.y, x[2] = a.z, x[3] = a.w;
  } else {
    for (int j = 0; j < 4; ++j) x[j] = (v0 + j < n) ? p[v0 + j] : 0;
  }
}

// k-out sampling: for every vertex with an edge, unite it with its first
// neighbour (hybrid, afforest) or a seeded pick (pure), then with k-1 more
// picks, using UF-Rem-CAS with SplitAtomicOne.  All picked neighbours of a
// vertex are loaded before its first union so their latencies overlap.
// Max-degree edge choice, before the unions: pick0[v] = row position of v's
// neighbour of largest degree (the first on ties).  Rows of at most
// kMaxdegLane entries are scanned by one lane; longer rows are listed and a
// wave per row scans them with a wave-wide maximum.
constexpr int kMaxdegLane = 64;

__device__ __forceinline__ unsigned long long maxdeg_key(int64_t deg, int64_t t) {
  // larger degree first, then smaller position
  return ((unsigned long long)deg << 32) | (unsigned long long)(0xffffffffu - (uint32_t)t);
}

template <typename I>
__global__ void __launch_bounds__(kBlock) k_maxdeg_short(int64_t n, const I* __restrict__ off,
                                                         const int32_t* __restrict__ adj, int32_t* __restrict__ pick0,
                                                         int32_t* __restrict__ longrows, int32_t* nlong) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    int64_t b = 0, deg = 0;
    if (v < n) {
      b = (int64_t)off[v];
      deg = (int64_t)off[v + 1] - b;
    }
    const bool lng = deg > kMaxdegLane;
    const uint64_t m = __ballot(lng);
    if (m) {
      const int leader = __ffsll((unsigned long long)m) - 1;
      int32_t pos = 0;
      if (lane_id() == leader) pos = atomicAdd(nlong, (int32_t)__popcll(m));
      pos = __shfl(pos, leader, kWave);
      if (lng) longrows[pos + __popcll(m & lanemask_lt_dev())] = (int32_t)v;
    }
    if (v >= n || deg <= 0 || lng) continue;
    unsigned long long best = 0;
    for (int64_t t = 0; t < deg; ++t) {
      const int32_t x = adj[b + t];
      const unsigned long long key = maxdeg_key((int64_t)off[x + 1] - (int64_t)off[x], t);
      best = key > best ? key : best;
    }
    pick0[v] = (int32_t)(0xffffffffu - (uint32_t)(best & 0xffffffffull));
  }
}

template <typename I>
__global__ void __launch_bounds__(kBlock) k_maxdeg_long(const I* __restrict__ off, const int32_t* __restrict__ adj,
                                                        const int32_t* __restrict__ longrows, const int32_t* nlong,
                                                        int32_t* __restrict__ pick0) {
  const int64_t c = *nlong;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < c; i += waves) {
    const int32_t v = longrows[i];
    const int64_t b = (int64_t)off[v];
    const int64_t deg = (int64_t)off[v + 1] - b;
    unsigned long long best = 0;
    for (int64_t t = lane_id(); t < deg; t += kWave) {
      const int32_t x = adj[b + t];
      const unsigned long long key = maxdeg_key((int64_t)off[x + 1] - (int64_t)off[x], t);
      best = key > best ? key : best;
    }
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long y = __shfl_xor(best, o, kWave);
      best = y > best ? y : best;
    }
    if (lane_id() == 0) pick0[v] = (int32_t)(0xffffffffu - (uint32_t)(best & 0xffffffffull));
  }
}

__global__ void k_zero_one_i32(int32_t* p) { *p = 0; }

// k-out's unions are UF-Rem-CAS with FindNaive and, by default,
// SplitAtomicOne.  When the whole graph is in flight at once (small n) and
// dense, splitting costs more than it saves: every split is a CAS on a
// parent slot near the top of a shared tree, which every other walk is
// reading, so those lines bounce between the CUs.  Then (dense_rule) a
// vertex of degree above kSplitDegree hooks without splitting; vertices of
// lower degree, which on lattices and chains hang in long paths, still
// split.  Both choices give the same partition.
constexpr int64_t kDenseRuleMaxN = (int64_t)1 << 20;
constexpr int64_t kSplitDegree = 4;

template <typename I>
__global__ void __launch_bounds__(kBlock) k_kout(int64_t n, const I* __restrict__ off, const int32_t* __restrict__ adj,
                                                 int32_t* P, int k, int mode, uint64_t key, int2* hook,
                                                 const int32_t* __restrict__ pick0, int32_t* __restrict__ count,
                                                 int dense_rule, int by_xcd) {
  constexpr int kMaxPreload = 4;
  const XcdSweep sw = by_xcd ? xcd_sweep(n)
                             : XcdSweep{(int64_t)blockIdx.x * blockDim.x, n, (int64_t)gridDim.x * blockDim.x};
  for (int64_t v = sw.base + threadIdx.x; v < sw.end; v += sw.step) {
    if (count) count[v] = 0;  // IdentifyFrequent's histogram, cleared here instead of by the init
    const int64_t b = (int64_t)off[v];
    const int64_t deg = (int64_t)off[v + 1] - b;
    if (deg <= 0) continue;
    const bool split = !dense_rule || deg <= kSplitDegree;
    int32_t w[kMaxPreload];
    const int kk = k < kMaxPreload ? k : kMaxPreload;
    int got = 0;
    for (int j = 0; j < kk; ++j) {
      int64_t idx;
      if (mode == CC_KOUT_AFFOREST) {
        if (j >= deg) break;
        idx = j;
      } else if (mode == CC_KOUT_HYBRID && j == 0) {
        idx = 0;
      } else if (mode == CC_KOUT_MAXDEG && j == 0) {
        idx = pick0[v];  // the neighbour of largest degree, the first one on ties
      } else {
        idx = (int64_t)(sm_out(key, (uint64_t)v * (uint64_t)k + (uint64_t)j) % (uint64_t)deg);
      }
      w[j] = adj[b + idx];
      got = j + 1;
    }
    for (int j = 0; j < got; ++j) forest_record(hook, union_rem_opt_split(P, (int32_t)v, w[j], split), (int32_t)v, w[j]);
    for (int j = kMaxPreload; j < k; ++j) {
      int64_t idx;
      if (mode == CC_KOUT_AFFOREST) {
        if (j >= deg) break;
        idx = j;
      } else {
        idx = (int64_t)(sm_out(key, (uint64_t)v * (uint64_t)k + (uint64_t)j) % (uint64_t)deg);
      }
      const int32_t w2 = adj[b + idx];
      forest_record(hook, union_rem_opt_split(P, (int32_t)v, w2, split), (int32_t)v, w2);
    }
  }
}

// Full compression fused with the IdentifyFrequent histogram.  Only vertices
// with at least one edge are counted (an isolated vertex is a class of its
// own and cannot be the unique most frequent one; if every class is a
// singleton, skipping nothing is equivalent).  Counting is aggregated twice:
// each wave peels its lanes into runs of equal labels (one add per run), and
// the block keeps the counts of up to kHotSlots labels in an LDS table
// (direct-mapped by label), so a few giant classes cost one global atomic
// per block each instead of one per vertex.
constexpr int kHotSlots = 32;

// Root of u in a forest that no union changes meanwhile (the compression
// sweep after the sampling).  The walk is naive for
// kSweepWalk steps, deeper than the trees of nearly every graph; past them
// it halves: each further node is pointed at its grandparent with a CAS (an
// ancestor either way, and a slot another lane has already changed is left
// alone), so lanes walking one long path (an id-ordered path graph) shorten
// it for each other instead of each walking all of it.
constexpr int kSweepWalk = 64;
__device__ __forceinline__ int32_t find_sweep(int32_t* P, int32_t u) {
  int32_t p = ld(P + u);
  for (int i = 0; i < kSweepWalk; ++i) {
    if (p == u) return u;
    u = p;
    p = ld(P + u);
  }
  while (p != u) {
    const int32_t g = ld(P + p);
    if (g != p) cas(P + u, p, g);
    u = g;
    p = ld(P + u);
  }
  return u;
}

template <typename I>
__global__ void __launch_bounds__(kBlock) k_compress_count(int64_t n, const I* __restrict__ off, int32_t* P,
                                                           int32_t* __restrict__ count, int2* __restrict__ hotpart,
                                                           int aligned) {
  __shared__ int32_t hot_label[kHotSlots];
  __shared__ int32_t hot_cnt[kHotSlots];
  if (threadIdx.x < kHotSlots) {
    hot_label[threadIdx.x] = -1;
    hot_cnt[threadIdx.x] = 0;
  }
  __syncthreads();
  const int lane = lane_id();
  const int64_t groups = div_up_dev(n, 4);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t gbase = blockIdx.x * (int64_t)blockDim.x; gbase < groups; gbase += stride) {
    const int64_t g = gbase + threadIdx.x;
    const int64_t v0 = 4 * g;
    int32_t p[4] = {0, 0, 0, 0};
    int64_t o[5] = {0, 0, 0, 0, 0};
    const bool act = g < groups;
    const bool vec = aligned && v0 + 3 < n;
    if (act) {
      load4(P, v0, vec, n, p);
      if (count) load_off5(off, v0, vec, n, o);
    }
    int32_t r[4];
    bool moved = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      r[j] = p[j];
      if (act && v0 + j < n && p[j] != (int32_t)(v0 + j)) {
        r[j] = find_sweep(P, p[j]);
        moved |= r[j] != p[j];
      }
    }
    // one 16-byte store for the lane's four slots (whole lines when most
    // lanes change, as after k-out on meshes); each slot is owned by this lane
    if (moved) {
      if (vec) {
        *(int4*)(P + v0) = make_int4(r[0], r[1], r[2], r[3]);
      } else {
        for (int j = 0; j < 4; ++j)
          if (act && v0 + j < n && r[j] != p[j]) st(P + v0 + j, r[j]);
      }
    }
    if (!count) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bool c = act && v0 + j < n && o[j + 1] > o[j];
      uint64_t mact = __ballot(c);
      while (mact) {
        const int leader = __ffsll((unsigned long long)mact) - 1;
        const int32_t lead = __shfl(r[j], leader, kWave);
        const uint64_t same = __ballot(c && r[j] == lead);
        if (lane == leader) {
          const int32_t add = (int32_t)__popcll(same);
          const int slot = (int)((uint32_t)lead % kHotSlots);
          int32_t h = hot_label[slot];
          if (h == -1) {
            atomicCAS(&hot_label[slot], -1, lead);
            h = hot_label[slot];
          }
          if (h == lead) atomicAdd(&hot_cnt[slot], add);
          else __hip_atomic_fetch_add(count + lead, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (r[j] == lead) c = false;
        mact &= ~same;
      }
    }
  }
  if (!count) return;
  __syncthreads();
  // Entries counted more than once in this block go to the block's own
  // slots of hotpart and a merge kernel adds them, so a class spread over
  // every block costs no address one atomic per block; single counts (small
  // classes, each touching few blocks) are added directly.
  if (threadIdx.x < kHotSlots) {
    const int32_t c = hot_cnt[threadIdx.x], lab = hot_label[threadIdx.x];
    const bool keep = c > 1;
    if (c == 1) __hip_atomic_fetch_add(count + lab, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    hotpart[(int64_t)blockIdx.x * kHotSlots + threadIdx.x] = make_int2(keep ? lab : -1, keep ? c : 0);
  }
}

// Adds the blocks' hot-table entries into count: block (s, c) walks slot s
// of blocks [256c, 256c + 256); a wave peels runs of equal labels and adds
// each run once.
__global__ void __launch_bounds__(kBlock) k_hot_merge(int nblocks, const int2* __restrict__ hotpart,
                                                      int32_t* __restrict__ count) {
  const int s = blockIdx.x % kHotSlots;
  {
    const int b = (blockIdx.x / kHotSlots) * kBlock + threadIdx.x;
    int2 e = make_int2(-1, 0);
    if (b < nblocks) e = hotpart[(int64_t)b * kHotSlots + s];
    bool c = e.x >= 0;
    uint64_t mact = __ballot(c);
    while (mact) {
      const int leader = __ffsll((unsigned long long)mact) - 1;
      const int32_t lead = __shfl(e.x, leader, kWave);
      const bool mine = c && e.x == lead;
      int32_t add = mine ? e.y : 0;
      for (int o = 32; o > 0; o >>= 1) add += __shfl_xor(add, o, kWave);
      if (lane_id() == leader) __hip_atomic_fetch_add(count + lead, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      mact &= ~__ballot(mine);
      if (mine) c = false;
    }
  }
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long y = __shfl_xor(x, o, kWave);
    x = y > x ? y : x;
  }
  return x;
}

__device__ __forceinline__ int32_t lmax_of(unsigned long long key) {
  return key ? (int32_t)(~(uint32_t)(key & 0xffffffffull)) : -1;
}

// Reduces nparts block maxima (nparts 0: no frequent label) and publishes
// lmax and its class size (one block).
__device__ __forceinline__ void resolve_lmax(DevScalars* sc, const unsigned long long* part, int nparts) {
  __shared__ unsigned long long red[kBlock / kWave];
  unsigned long long best = 0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) best = part[i] > best ? part[i] : best;
  best = wave_max_u64(best);
  if (lane_id() == 0) red[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) best = red[w] > best ? red[w] : best;
    sc->lmax_key = best;
    sc->lmax = lmax_of(best);
    sc->lmax_size = (long long)(best >> 32);
  }
}

// IdentifyFrequent: max over (count << 32 | ~label); ties go to the smaller
// label.  Each block writes its maximum to part[blockIdx]; one block
// reduces them (no address takes an atomic per block).  A last-block
// reduction inside this kernel was measured slower: the agent-scope fence
// each block needs before its ticket writes back its XCD's L2.
__global__ void __launch_bounds__(kBlock) k_argmax(int64_t n, const int32_t* __restrict__ count,
                                                   unsigned long long* __restrict__ part, int aligned) {
  __shared__ unsigned long long red[kBlock / kWave];
  unsigned long long best = 0;
  const int64_t groups = div_up_dev(n, 4);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < groups; g += stride) {
    const int64_t v0 = 4 * g;
    int32_t c[4];
    load4(count, v0, aligned && v0 + 3 < n, n, c);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (c[j] > 0 && v0 + j < n) {
        const unsigned long long key = ((unsigned long long)(uint32_t)c[j] << 32) | (uint32_t)(~(uint32_t)(v0 + j));
        best = key > best ? key : best;
      }
  }
  best = wave_max_u64(best);
  if (lane_id() == 0) red[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) best = red[w] > best ? red[w] : best;
    part[blockIdx.x] = best;
  }
}

__global__ void __launch_bounds__(kBlock) k_resolve_lmax(DevScalars* sc, const unsigned long long* __restrict__ part,
                                                         int nparts) {
  resolve_lmax(sc, part, nparts);
}

// Candidate compaction with degree binning, in three launches and without
// contended atomics.  Wave w owns the vertex range [w*S, min((w+1)*S, n)) and
// the same range of the scratch array: thread-bin candidates (degree <=
// kThrWave) fill it from the front, all others from the back.  A one-block
// scan turns the per-wave counts of the four bins into list offsets, and a
// gather copies every segment into the final lists (thread bin: cand; wave
// bin: big front; block bin: big back; grid bin: heavy), classifying the
// back entries by degree.  The lists come out in a fixed order, so the finish
// does the same work every run.  The scan is two-level: each block of the
// segment kernel (four waves, four consecutive segments) also writes its
// group's totals, the one-block scan runs over groups only, and the gather
// adds the counts of the at most three earlier segments of its group.  The
// grid bin's degree prefix (the offsets its edge-balanced visitor searches)
// is built along the way: per-segment sums of the grid-bin degrees, scanned
// with the counts, then a wave scan in the gather.
constexpr int kSegMax = 8448;  // upper bound on the number of segments

template <typename I>
__global__ void __launch_bounds__(kBlock) k_compact_seg(int64_t n, int64_t S, const I* __restrict__ off,
                                                        const int32_t* __restrict__ P, const DevScalars* sc,
                                                        int32_t* __restrict__ scratch, int32_t* __restrict__ segcnt,
                                                        long long* __restrict__ segedges,
                                                        long long* __restrict__ segheavy,
                                                        int4* __restrict__ grpcnt, long long* __restrict__ grpedges,
                                                        long long* __restrict__ grpheavy, int aligned) {
  static_assert(kBlock / kWave == 4, "a block is one group of four segments");
  __shared__ int32_t gc[4][4];
  __shared__ long long ge[4], gh[4];
  const int32_t L = sc->lmax;
  const int lane = lane_id();
  const int wv = threadIdx.x / kWave;
  const uint64_t lt = lanemask_lt_dev();
  const int64_t nseg = div_up_dev(n, S);
  const int64_t w = blockIdx.x * (int64_t)(blockDim.x / kWave) + wv;  // one segment per wave
  int32_t c0 = 0, cb = 0, c2 = 0, c3 = 0;
  long long edges = 0, hedges = 0;
  if (w < nseg) {
    const int64_t lo = w * S;
    const int64_t hi = (lo + S < n) ? lo + S : n;
    for (int64_t base = lo; base < hi; base += 4 * kWave) {
      const int64_t v0 = base + 4 * lane;
      const bool act = v0 < hi;
      const bool vec = aligned && v0 + 3 < hi;
      int32_t p[4] = {0, 0, 0, 0};
      int64_t o[5] = {0, 0, 0, 0, 0};
      if (act) {
        load4(P, v0, vec, n, p);
        load_off5(off, v0, vec, n, o);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool inb = act && v0 + j < hi;
        const int64_t deg = inb ? o[j + 1] - o[j] : 0;
        const bool isc = inb && deg > 0 && p[j] != L;
        if (isc) edges += deg;
        const bool small = isc && deg <= kThrWave;
        const bool large = isc && deg > kThrWave;
        const uint64_t ms = __ballot(small);
        const uint64_t ml = __ballot(large);
        if (small) scratch[lo + c0 + __popcll(ms & lt)] = (int32_t)(v0 + j);
        if (large) scratch[hi - 1 - (cb + __popcll(ml & lt))] = (int32_t)(v0 + j);
        c0 += __popcll(ms);
        cb += __popcll(ml);
        c2 += __popcll(__ballot(large && deg > kThrBlock && deg <= kThrGrid));
        c3 += __popcll(__ballot(large && deg > kThrGrid));
        if (large && deg > kThrGrid) hedges += deg;
      }
    }
  }
  edges = wave_sum(edges);
  hedges = wave_sum(hedges);
  if (lane == 0) {
    if (w < nseg) {
      *(int4*)(segcnt + 4 * w) = make_int4(c0, cb - c2 - c3, c2, c3);
      segedges[w] = edges;
      segheavy[w] = hedges;
    }
    gc[wv][0] = c0, gc[wv][1] = cb - c2 - c3, gc[wv][2] = c2, gc[wv][3] = c3;
    ge[wv] = edges;
    gh[wv] = hedges;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int4 t = make_int4(0, 0, 0, 0);
    long long e = 0, h = 0;
    for (int k = 0; k < 4; ++k) {
      t.x += gc[k][0], t.y += gc[k][1], t.z += gc[k][2], t.w += gc[k][3];
      e += ge[k];
      h += gh[k];
    }
    grpcnt[blockIdx.x] = t;
    grpedges[blockIdx.x] = e;
    grpheavy[blockIdx.x] = h;
  }
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int lane = lane_id();
  for (int o = 1; o < kWave; o <<= 1) {
    const T y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  return x;
}

// One block: exclusive scan of the group totals (four bin counts and the
// grid-bin degree sums), in place; bin totals and the candidates' edge total
// into the context scalars, the grid bin's edge total into hp[count].
// Thread t owns a run of at most kScanRun consecutive groups, loaded all at
// once; the run totals go through one block scan (wave scans, then one wave
// scans the wave totals), and each thread writes its run back.
constexpr int kGrpMax = kSegMax / 4;
constexpr int kScanRun = (kGrpMax + 1023) / 1024;

__global__ void __launch_bounds__(1024) k_compact_scan(int64_t ngrp, int4* grpcnt, const long long* grpedges,
                                                       long long* grpheavy, long long* hp, DevScalars* sc) {
  constexpr int kWaves = 1024 / kWave;
  __shared__ int32_t wc[4][kWaves];
  __shared__ long long wh[kWaves];
  __shared__ long long we[kWaves];
  __shared__ int32_t tot[4];
  __shared__ long long htot;
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  const int64_t per = div_up_dev(ngrp, 1024);
  const int64_t lo = t * per;
  int4 c[kScanRun];
  long long h[kScanRun];
  int32_t sum[4] = {0, 0, 0, 0};
  long long hs = 0, e = 0;
#pragma unroll
  for (int j = 0; j < kScanRun; ++j) {
    const int64_t i = lo + j;
    c[j] = make_int4(0, 0, 0, 0);
    h[j] = 0;
    if (j < per && i < ngrp) {
      c[j] = grpcnt[i];
      h[j] = grpheavy[i];
      e += grpedges[i];
    }
  }
#pragma unroll
  for (int j = 0; j < kScanRun; ++j) {
    sum[0] += c[j].x, sum[1] += c[j].y, sum[2] += c[j].z, sum[3] += c[j].w;
    hs += h[j];
  }
  int32_t inc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) inc[q] = wave_incl_scan(sum[q]);
  const long long hinc = wave_incl_scan(hs);
  e = wave_sum(e);
  if (lane == kWave - 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) wc[q][w] = inc[q];
    wh[w] = hinc;
  }
  if (lane == 0) we[w] = e;
  __syncthreads();
  if (w == 0) {  // exclusive scan of the wave totals by one wave
    const bool in = lane < kWaves;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int32_t x = in ? wc[q][lane] : 0;
      const int32_t y = wave_incl_scan(x);
      if (in) wc[q][lane] = y - x;
      if (lane == kWaves - 1) tot[q] = y;
    }
    const long long x = in ? wh[lane] : 0;
    const long long y = wave_incl_scan(x);
    if (in) wh[lane] = y - x;
    if (lane == kWaves - 1) htot = y;
  }
  __syncthreads();
  int32_t r[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = wc[q][w] + inc[q] - sum[q];
  long long hr = wh[w] + hinc - hs;
#pragma unroll
  for (int j = 0; j < kScanRun; ++j) {
    const int64_t i = lo + j;
    if (j < per && i < ngrp) {
      grpcnt[i] = make_int4(r[0], r[1], r[2], r[3]);
      grpheavy[i] = hr;
      r[0] += c[j].x, r[1] += c[j].y, r[2] += c[j].z, r[3] += c[j].w;
      hr += h[j];
    }
  }
  if (t == 0) {
    long long et = 0;
    for (int k = 0; k < kWaves; ++k) et += we[k];
    sc->cand_edges = et;
    for (int q = 0; q < 4; ++q) sc->bin_count[q] = tot[q];
    hp[tot[3]] = htot;  // the grid bin's edge total closes its prefix
  }
}

template <typename I>
__global__ void __launch_bounds__(kBlock) k_compact_gather(int64_t n, int64_t S, const I* __restrict__ off,
                                                           const int32_t* __restrict__ scratch,
                                                           const int4* __restrict__ segcnt,
                                                           const long long* __restrict__ segheavy,
                                                           const int4* __restrict__ grpoff,
                                                           const long long* __restrict__ grpheavy,
                                                           int32_t* __restrict__ cand, int32_t* __restrict__ big,
                                                           int32_t* __restrict__ heavy, long long* __restrict__ hp) {
  const int lane = lane_id();
  const uint64_t lt = lanemask_lt_dev();
  const int64_t nseg = div_up_dev(n, S);
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t w = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; w < nseg; w += waves) {
    const int64_t lo = w * S;
    const int64_t hi = (lo + S < n) ? lo + S : n;
    // this segment's list offsets: its group's offsets plus the counts of
    // the group's earlier segments
    const int64_t g = w / 4;
    int4 ov = grpoff[g];
    long long hb = grpheavy[g];
    for (int64_t s2 = 4 * g; s2 < w; ++s2) {
      const int4 x = segcnt[s2];
      ov.x += x.x, ov.y += x.y, ov.z += x.z, ov.w += x.w;
      hb += segheavy[s2];
    }
    const int4 cv = segcnt[w];
    const int32_t o[4] = {ov.x, ov.y, ov.z, ov.w};
    const int32_t c[4] = {cv.x, cv.y, cv.z, cv.w};
    for (int32_t i = lane; i < c[0]; i += kWave) cand[o[0] + i] = scratch[lo + i];
    const int32_t cb = c[1] + c[2] + c[3];
    int32_t r1 = o[1], r2 = o[2], r3 = o[3];
    for (int32_t i0 = 0; i0 < cb; i0 += kWave) {
      const int32_t i = i0 + lane;
      int32_t x = 0;
      int64_t deg = 0;
      if (i < cb) {
        x = scratch[hi - 1 - i];
        deg = (int64_t)off[x + 1] - (int64_t)off[x];
      }
      const bool b1 = i < cb && deg <= kThrBlock;
      const bool b2 = i < cb && deg > kThrBlock && deg <= kThrGrid;
      const bool b3 = i < cb && deg > kThrGrid;
      const uint64_t m1 = __ballot(b1), m2 = __ballot(b2), m3 = __ballot(b3);
      if (b1) big[r1 + __popcll(m1 & lt)] = x;
      if (b2) big[n - 1 - (r2 + __popcll(m2 & lt))] = x;
      if (m3) {  // grid bin: row and its degree prefix
        const long long hd = b3 ? deg : 0;
        const long long hinc = wave_incl_scan(hd);
        if (b3) {
          heavy[r3 + __popcll(m3 & lt)] = x;
          hp[r3 + __popcll(m3 & lt)] = hb + hinc - hd;
        }
        hb += __shfl(hinc, kWave - 1, kWave);
      }
      r1 += __popcll(m1);
      r2 += __popcll(m2);
      r3 += __popcll(m3);
    }
  }
}

// Union-find finish operator: Union(u, w) with the variant's rules.
template <int ALG, int SPLICE, int FIND>
struct UnionOp {
  int32_t* P;
  int2* hook;   // spanning forest: edge per hooked root (nullable)
  int32_t* H;   // UF-Hooks: claim array (else unused)
  __device__ __forceinline__ bool operator()(int32_t u, int32_t w, int64_t) const {
    forest_record(hook, unite<ALG, SPLICE, FIND>(P, u, w, H), u, w);
    return false;
  }
};

// Final compression and component count: label = root (the component's
// minimum, since every link points to a smaller id).  Per-block root counts
// go to part[].
// With orig_of (a renumbered CSR), the sweep also copies each root's
// original id into rmin, the start of its minimum original id (see
// k_map_min).
__global__ void __launch_bounds__(kBlock) k_output(int64_t n, int32_t* P, long long* __restrict__ part,
                                                   int aligned, const int32_t* __restrict__ orig_of,
                                                   int32_t* __restrict__ rmin) {
  __shared__ long long red[kBlock / kWave];
  long long roots = 0;
  const int64_t groups = div_up_dev(n, 4);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < groups; g += stride) {
    const int64_t v0 = 4 * g;
    const bool vec = aligned && v0 + 3 < n;
    int32_t p[4], r[4];
    load4(P, v0, vec, n, p);
    if (orig_of) {
      // only a root's slot is ever read, so groups without one skip the copy
      // (most of them, where the non-isolated vertices come first)
      if (vec) {
        if (p[0] == (int32_t)v0 || p[1] == (int32_t)(v0 + 1) || p[2] == (int32_t)(v0 + 2) ||
            p[3] == (int32_t)(v0 + 3))
          *(int4*)(rmin + v0) = *(const int4*)(orig_of + v0);
      } else {
        for (int j = 0; j < 4; ++j)
          if (v0 + j < n && p[j] == (int32_t)(v0 + j)) rmin[v0 + j] = orig_of[v0 + j];
      }
    }
    bool moved = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t v = v0 + j;
      r[j] = p[j];
      if (v >= n) continue;
      if (p[j] == (int32_t)v) {
        ++roots;
        continue;
      }
      r[j] = find_naive(P, p[j]);
      moved |= r[j] != p[j];
    }
    if (moved) {
      if (vec) {
        *(int4*)(P + v0) = make_int4(r[0], r[1], r[2], r[3]);
      } else {
        for (int j = 0; j < 4; ++j)
          if (v0 + j < n && r[j] != p[j]) st(P + v0 + j, r[j]);
      }
    }
  }
  roots = wave_sum(roots);
  if (lane_id() == 0) red[threadIdx.x / kWave] = roots;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) roots += red[w];
    part[blockIdx.x] = roots;
  }
}

// ---- labels in the original numbering -----------------------------------
// For a CSR whose vertices were renumbered (orig_of[x] = the original id of
// vertex x, new_of its inverse), the labels come out in the new numbering
// (each component's smallest new id); the caller wants each original vertex
// labelled with its component's smallest original id.  rmin[r] collects
// that minimum for every root r: it starts as the root's own original id
// (copied by the output sweep), every other vertex adds its own with
// atomicMin, and the vertices of the
// frequent class's component (root P[lmax]; most of a power-law graph) fold
// theirs into one partial per block instead, so that no address takes one
// atomic per vertex.  A gather then labels the original vertices from the
// tail and the frequent component, and a pass over the frequent component's
// bitmap corrects the rest.
__device__ __forceinline__ int32_t wave_min_i32(int32_t v) {
  for (int o = 32; o > 0; o >>= 1) {
    const int32_t y = __shfl_xor(v, o, kWave);
    v = y < v ? y : v;
  }
  return v;
}

__global__ void __launch_bounds__(kBlock) k_map_min(int64_t n, const int32_t* __restrict__ P,
                                                    const int32_t* __restrict__ orig_of, int32_t* rmin,
                                                    const DevScalars* sc, int32_t* __restrict__ part,
                                                    uint32_t* __restrict__ in_giant, int aligned) {
  __shared__ int32_t red[kBlock / kWave];
  const int32_t L = sc->lmax;
  const int32_t Rg = L >= 0 ? P[L] : -1;
  int32_t bmin = 0x7fffffff;
  const int lane = lane_id();
  const int64_t groups = div_up_dev(n, 4);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // four consecutive vertices per lane, so a wave covers 256 vertices: eight
  // bitmap words, word j of the wave holding the nibbles of lanes 8j .. 8j + 7
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < groups; base += stride) {
    const int64_t g = base + threadIdx.x;
    const int64_t v0 = 4 * g;
    const bool vec = aligned && v0 + 3 < n;
    int32_t r[4], o[4] = {0x7fffffff, 0x7fffffff, 0x7fffffff, 0x7fffffff};
    bool nonroot[4];
    if (g < groups) {
      load4(P, v0, vec, n, r);
    } else {
      r[0] = r[1] = r[2] = r[3] = -1;
    }
    bool any = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      nonroot[j] = v0 + j < n && r[j] != (int32_t)(v0 + j);
      any |= nonroot[j];
    }
    if (any) load4(orig_of, v0, vec, n, o);
    uint32_t word = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (v0 + j < n && r[j] == Rg) word |= 1u << (4 * (lane & 7) + j);
      if (nonroot[j] && r[j] == Rg) bmin = o[j] < bmin ? o[j] : bmin;
    }
    word |= __shfl_xor(word, 1, kWave);
    word |= __shfl_xor(word, 2, kWave);
    word |= __shfl_xor(word, 4, kWave);
    const int64_t w = (base + (threadIdx.x & ~(kWave - 1))) / 8 + (lane >> 3);
    if ((lane & 7) == 0 && (w << 5) < n) in_giant[w] = word;
    // the other components: lanes with equal roots add one minimum per root
    // and wave
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bool act = nonroot[j] && r[j] != Rg;
      uint64_t mask = __ballot(act);
      while (mask) {
        const int leader = __ffsll((unsigned long long)mask) - 1;
        const int32_t lr = __shfl(r[j], leader, kWave);
        const bool mine = act && r[j] == lr;
        const int32_t mn = wave_min_i32(mine ? o[j] : 0x7fffffff);
        if (lane == leader) atomicMin(rmin + lr, mn);
        mask &= ~__ballot(mine);
        if (mine) act = false;
      }
    }
  }
  bmin = wave_min_i32(bmin);
  if (lane == 0) red[threadIdx.x / kWave] = bmin;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) bmin = red[w] < bmin ? red[w] : bmin;
    part[blockIdx.x] = bmin;
  }
}

// One block: the frequent component's minimum from the block partials, and
// the first vertex of the CSR's run of trailing empty rows (each of those
// vertices is alone in its component; a CSR in decreasing-degree order keeps
// every isolated vertex there).  The caller promised that rows na .. n-1
// are empty: the run starts at na unless row na-1 is empty too (then a
// binary search below na finds it); a broken promise sets the bad-CSR bit.
template <typename I>
__global__ void __launch_bounds__(kBlock) k_map_giant(int64_t n, int64_t na, const I* __restrict__ off,
                                                      const int32_t* __restrict__ P, DevScalars* sc,
                                                      const int32_t* __restrict__ part, int nparts, int32_t* rmin) {
  __shared__ int32_t red[kBlock / kWave];
  if (threadIdx.x == 0) {
    const I m = off[n];
    if (off[na] != m) {
      atomicOr(&sc->error, kErrBadCsr);
      sc->map_tail = na;
    } else if (na > 0 && off[na - 1] != m) {
      sc->map_tail = na;
    } else {
      int64_t lo = 0, hi = na;  // first x with off[x] == m (off[na] == m)
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (off[mid] == m) hi = mid;
        else lo = mid + 1;
      }
      sc->map_tail = lo;
    }
  }
  const int32_t L = sc->lmax;
  if (L < 0) return;
  int32_t m = 0x7fffffff;
  for (int i = threadIdx.x; i < nparts; i += kBlock) m = part[i] < m ? part[i] : m;
  m = wave_min_i32(m);
  if (lane_id() == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) m = red[w] < m ? red[w] : m;
    const int32_t Rg = P[L];
    if (m < rmin[Rg]) rmin[Rg] = m;
  }
}

// Original vertex o: its own id when its row lies in the trailing run of
// empty rows, else the frequent component's minimum.  Sequential reads and
// writes only; the vertices before the tail that are not in the frequent
// component are corrected by k_map_fix afterwards.
__global__ void __launch_bounds__(kBlock) k_map_gather(int64_t n, const int32_t* __restrict__ P,
                                                       const int32_t* __restrict__ new_of,
                                                       const int32_t* __restrict__ rmin, const DevScalars* sc,
                                                       int32_t* __restrict__ out, int aligned) {
  const int32_t L = sc->lmax;
  const int32_t gmin = L >= 0 ? rmin[P[L]] : 0;
  const int64_t tail = sc->map_tail;
  const int64_t groups = div_up_dev(n, 4);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < groups; g += stride) {
    const int64_t o0 = 4 * g;
    if (aligned && o0 + 3 < n) {
      const int4 x = *(const int4*)(new_of + o0);
      *(int4*)(out + o0) = make_int4(x.x >= tail ? (int32_t)o0 : gmin, x.y >= tail ? (int32_t)(o0 + 1) : gmin,
                                     x.z >= tail ? (int32_t)(o0 + 2) : gmin, x.w >= tail ? (int32_t)(o0 + 3) : gmin);
    } else {
      for (int64_t o = o0; o < n && o < o0 + 4; ++o) out[o] = new_of[o] >= tail ? (int32_t)o : gmin;
    }
  }
}

// Vertices x before the tail whose bit is clear (not in the frequent
// component, or an isolated vertex when the numbering leaves empty rows
// before the tail): their original vertex takes its root's minimum, which
// for an isolated root is its own original id.  One lane per bitmap word;
// when almost every vertex with an edge is in the frequent component (R-MAT)
// this touches a few thousand vertices, so the per-vertex random reads of
// the parent array leave the gather.
__global__ void __launch_bounds__(kBlock) k_map_fix(int64_t n, const int32_t* __restrict__ P,
                                                    const int32_t* __restrict__ orig_of,
                                                    const int32_t* __restrict__ rmin, const DevScalars* sc,
                                                    const uint32_t* __restrict__ in_giant, int32_t* out) {
  const int64_t tail = sc->map_tail < n ? sc->map_tail : n;
  const int64_t words = (tail + 31) >> 5;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < words; w += stride) {
    uint32_t need = ~in_giant[w];
    const int64_t x0 = w << 5;
    if (tail - x0 < 32) need &= (1u << (tail - x0)) - 1u;
    while (need) {
      const int64_t x = x0 + __builtin_ctz(need);
      need &= need - 1u;
      out[orig_of[x]] = rmin[P[x]];
    }
  }
}

// Component count from the per-block root counts (one block), plus `extra`
// isolated vertices outside the swept range.
__global__ void __launch_bounds__(kBlock) k_output_sum(const long long* __restrict__ part, int nparts, long long extra,
                                                       DevScalars* sc, long long* ncomp_user) {
  __shared__ long long red[kBlock / kWave];
  long long s = 0;
  for (int i = threadIdx.x; i < nparts; i += kBlock) s += part[i];
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) s += red[w];
    s += extra;
    sc->num_components = s;
    if (ncomp_user) *ncomp_user = s;
  }
}

// ---------------------------------------------------------------------------
// host orchestration

template <int ALG, int SPLICE, int FIND, typename I>
static cc_status launch_uf_finish(StaticArgs& a) {
  int32_t* H = nullptr;
  if (ALG == 3) {  // UF-Hooks: claims in the count array (free once the compaction ran)
    H = a.count;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(a.n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, (uint32_t*)H, a.n,
                       0xffffffffu);
  }
  visit_candidates(a.s, a.lists(), (const I*)a.off, a.adj, UnionOp<ALG, SPLICE, FIND>{a.P, a.hook_e, H},
                   (uint32_t*)nullptr);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

template <typename I>
static cc_status uf_finish_dispatch(StaticArgs& a) {
  const cc_variant* v = a.v;
  if (v->finish == CC_FIN_UF_REM_CAS) {
#define REM(SPL, FND)                                          \
  if (v->splice == SPL && v->find == FND) return launch_uf_finish<0, SPL, FND, I>(a);
    REM(0, 0) REM(0, 1) REM(0, 2) REM(1, 0) REM(1, 1) REM(1, 2) REM(2, 0) REM(2, 1) REM(2, 2)
#undef REM
  } else {
#define FINDS(ALG)                                                        \
  if (v->find == 0) return launch_uf_finish<ALG, 0, 0, I>(a);             \
  if (v->find == 1) return launch_uf_finish<ALG, 0, 1, I>(a);             \
  if (v->find == 2) return launch_uf_finish<ALG, 0, 2, I>(a);             \
  if (v->find == 3) return launch_uf_finish<ALG, 0, 3, I>(a);
    if (v->finish == CC_FIN_UF_ASYNC) {
      FINDS(1)
    } else if (v->finish == CC_FIN_UF_EARLY) {
      FINDS(2)
    } else if (v->finish == CC_FIN_UF_HOOKS) {
      FINDS(3)
    }
#undef FINDS
  }
  return fail(CC_EINVAL, "no such union-find variant");
}

static inline bool al16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
// Every array the streaming kernels read four-at-a-time is 16-byte aligned.
static inline int vec_ok(const StaticArgs& a) { return al16(a.P) && al16(a.off) && al16(a.count); }
static inline unsigned grid4(int64_t n) { return grid_for(div_up(n, 4), kBlock, 2048); }

template <typename I>
cc_status compress_count_frequent(StaticArgs& a, bool use_lmax) {
  const int vec = vec_ok(a);
  {
    PhaseScope ps(a.ctx, a.s, "compress_count");
    // per-block hot-table entries: kHotSlots int2 per block, in the
    // candidate array (unused until compaction; large enough for any n)
    int2* hotpart = (int2*)a.cand;
    const unsigned nb = grid4(a.n);
    hipLaunchKernelGGL(k_compress_count<I>, dim3(nb), dim3(kBlock), 0, a.s, a.n, (const I*)a.off, a.P,
                       use_lmax ? a.count : (int32_t*)nullptr, hotpart, vec);
    if (use_lmax)
      hipLaunchKernelGGL(k_hot_merge, dim3(kHotSlots * div_up(nb, kBlock)), dim3(kBlock), 0, a.s, (int)nb,
                         (const int2*)hotpart, a.count);
  }
  {
    PhaseScope ps(a.ctx, a.s, "frequent");
    // block maxima in the compaction area (unused until compaction)
    unsigned long long* part = (unsigned long long*)(a.ws + a.L.seg);
    const unsigned nb = grid4(a.n);
    if (use_lmax)
      hipLaunchKernelGGL(k_argmax, dim3(nb), dim3(kBlock), 0, a.s, a.n, (const int32_t*)a.count, part, vec);
    hipLaunchKernelGGL(k_resolve_lmax, dim3(1), dim3(kBlock), 0, a.s, a.ctx->dev, (const unsigned long long*)part,
                       use_lmax ? (int)nb : 0);
  }
  CC_LAUNCH_CHECK();
  return CC_OK;
}

template <typename I>
static cc_status run_sample(StaticArgs& a) {
  const cc_variant* v = a.v;
  a.sample_success = 1;
  a.sample_rounds = 0;
  bool use_lmax = false;
  switch (v->sample) {
    case CC_SAMPLE_NONE:
      a.sample_success = -1;
      break;
    case CC_SAMPLE_KOUT: {
      PhaseScope ps(a.ctx, a.s, "sample");
      const uint64_t key = sm_out(v->seed, kTagKout);
      int32_t* pick0 = nullptr;
      if (v->kout_mode == CC_KOUT_MAXDEG) {
        // pick positions in the candidate array, the long rows in the
        // big array, their count in a spare scalar (all free until the
        // compaction)
        pick0 = a.cand;
        int32_t* nlong = &a.ctx->dev->hcount;
        hipLaunchKernelGGL(k_zero_one_i32, dim3(1), dim3(1), 0, a.s, nlong);
        hipLaunchKernelGGL(k_maxdeg_short<I>, dim3(grid_for(a.n, kBlock, kStreamGridCap)), dim3(kBlock), 0, a.s, a.n,
                           (const I*)a.off, a.adj, pick0, a.big, nlong);
        hipLaunchKernelGGL(k_maxdeg_long<I>, dim3(2048), dim3(kBlock), 0, a.s, (const I*)a.off, a.adj,
                           (const int32_t*)a.big, (const int32_t*)nlong, pick0);
      }
      // one vertex per thread, each XCD on its own eighth of the ids: the
      // hardware spreads the blocks over the CUs as they free up, balancing
      // rows of different cost, and the unions of one XCD stay within its
      // range (R-MAT 2^24: grid-stride 0.53, one per thread 0.49, by XCD
      // 0.47 ms; 256^3 grid: 1.00, 1.38, 1.07 ms)
      // (A CSR renumbered by decreasing degree runs its blocks in id order
      // instead: there the ranges would be unequal work, the hubs in the
      // first and the isolated vertices in the last.)
      // Sparse graphs (m < 3n: lattices, chains) run 2048 blocks striding
      // through their XCD's range instead of one vertex per thread: fewer
      // neighbouring vertices hook at the same moment (256^3 grid 1.07 ->
      // 0.84 ms; R-MAT 2^24 would lose, 0.47 -> 0.61 ms).
      const int64_t kcap = a.m < 3 * a.n ? 2048 : kVertexGridCap;
      hipLaunchKernelGGL(k_kout<I>,
                         dim3(a.kout_by_xcd ? xcd_grid(a.n, kBlock, kcap) : grid_for(a.n, kBlock, kVertexGridCap)),
                         dim3(kBlock), 0, a.s, a.n, (const I*)a.off, a.adj, a.P, v->kout_k, v->kout_mode, key,
                         a.hook_e, (const int32_t*)pick0, a.count, (int)(a.n <= kDenseRuleMaxN && a.m >= 3 * a.n),
                         (int)a.kout_by_xcd);
      CC_LAUNCH_CHECK();
      use_lmax = true;
      break;
    }
    case CC_SAMPLE_BFS: {
      cc_status st;
      {
        PhaseScope ps(a.ctx, a.s, "sample");
        st = sample_bfs<I>(a);
      }
      if (st != CC_OK) return st;
      use_lmax = a.sample_success >= 0;
      break;
    }
    case CC_SAMPLE_LDD: {
      cc_status st;
      {
        PhaseScope ps(a.ctx, a.s, "sample");
        st = sample_ldd<I>(a);
      }
      if (st != CC_OK) return st;
      use_lmax = true;
      break;
    }
  }
  return compress_count_frequent<I>(a, use_lmax);
}

template <typename I>
static cc_status run_tail(StaticArgs& a);

template <typename I>
static cc_status run_static(StaticArgs& a, bool sample_only) {
  if (!a.skip_init) {
    PhaseScope ps(a.ctx, a.s, "init");
    // no sampling needs no histogram; k-out clears it in its own sweep
    const bool no_count = a.v->sample == CC_SAMPLE_NONE || a.v->sample == CC_SAMPLE_KOUT;
    const int64_t np = a.n_parents > a.n ? a.n_parents : a.n;
    hipLaunchKernelGGL(k_init, dim3(grid4(np)), dim3(kBlock), 0, a.s, a.n, np, a.P,
                       no_count ? (int32_t*)nullptr : a.count, vec_ok(a), a.ctx->dev, (long long*)a.ncomp_user);
    CC_LAUNCH_CHECK();
  }
  cc_status st = run_sample<I>(a);
  if (st != CC_OK || sample_only) return st;
  return run_tail<I>(a);
}

// Candidate lists of the vertices outside the frequent label (resolved in
// the context scalars), binned by degree.
template <typename I>
cc_status compact_candidates(StaticArgs& a) {
  PhaseScope ps(a.ctx, a.s, "compact");
  // segment size: a multiple of 256 vertices, at most ~8192 segments
  int64_t S = div_up(div_up(a.n, 8192), 256) * 256;
  const int64_t nseg = div_up(a.n, S);
  int32_t* segcnt = (int32_t*)(a.ws + a.L.seg);
  long long* segedges = (long long*)(a.ws + a.L.seg + align256((size_t)kSegMax * 16));
  long long* segheavy = segedges + align256((size_t)kSegMax * 8) / 8;
  int4* grpcnt = (int4*)(segheavy + align256((size_t)kSegMax * 8) / 8);
  long long* grpedges = (long long*)(grpcnt + align256((size_t)kGrpMax * 16) / 16);
  long long* grpheavy = grpedges + align256((size_t)kGrpMax * 8) / 8;
  // one block per group of four segments; the gather walks the segments
  const int64_t ngrp = div_up(nseg, 4);
  const unsigned gw = (unsigned)ngrp;
  hipLaunchKernelGGL(k_compact_seg<I>, dim3(gw), dim3(kBlock), 0, a.s, a.n, S, (const I*)a.off,
                     (const int32_t*)a.P, (const DevScalars*)a.ctx->dev, a.count, segcnt, segedges, segheavy,
                     grpcnt, grpedges, grpheavy, vec_ok(a));
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, a.s, ngrp, grpcnt, (const long long*)grpedges,
                     grpheavy, a.hp, a.ctx->dev);
  hipLaunchKernelGGL(k_compact_gather<I>, dim3(gw), dim3(kBlock), 0, a.s, a.n, S, (const I*)a.off,
                     (const int32_t*)a.count, (const int4*)segcnt, (const long long*)segheavy,
                     (const int4*)grpcnt, (const long long*)grpheavy, a.cand, a.big, a.heavy, a.hp);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

template <typename I>
cc_status prepare_candidates(StaticArgs& a) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(a.n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, (uint32_t*)a.count,
                     a.n, 0u);
  cc_status st = compress_count_frequent<I>(a, true);
  if (st != CC_OK) return st;
  return compact_candidates<I>(a);
}
template cc_status prepare_candidates<int32_t>(StaticArgs&);
template cc_status prepare_candidates<int64_t>(StaticArgs&);

cc_status output_labels(StaticArgs& a) {
  PhaseScope ps(a.ctx, a.s, "output");
  // per-block root counts in the compaction area (free once the finish ran)
  long long* part = (long long*)(a.ws + a.L.seg);
  const unsigned nb = grid4(a.n);
  const int vec = vec_ok(a) && (!a.map_orig || (al16(a.map_orig) && al16(a.map_rmin)));
  hipLaunchKernelGGL(k_output, dim3(nb), dim3(kBlock), 0, a.s, a.n, a.P, part, vec, a.map_orig, a.map_rmin);
  const long long extra = a.n_parents > a.n ? (long long)(a.n_parents - a.n) : 0;
  hipLaunchKernelGGL(k_output_sum, dim3(1), dim3(kBlock), 0, a.s, (const long long*)part, (int)nb, extra,
                     a.ctx->dev, (long long*)a.ncomp_user);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

// Compaction, finish and output, on a parent array that already holds a
// sampled labelling with its frequent label resolved in the context scalars.
template <typename I>
static cc_status run_tail(StaticArgs& a) {
  cc_status st = compact_candidates<I>(a);
  if (st != CC_OK) return st;
  a.finish_rounds = 0;
  {
    PhaseScope ps(a.ctx, a.s, "finish");
    if (a.v->finish == CC_FIN_SV) st = finish_sv<I>(a);
    else if (a.v->finish == CC_FIN_LT) st = finish_lt<I>(a);
    else if (a.v->finish == CC_FIN_LP) st = finish_lp<I>(a);
    else st = uf_finish_dispatch<I>(a);
  }
  if (st != CC_OK) return st;
  return output_labels(a);
}


static void record_stats_host(StaticArgs& a);

cc_status static_init(StaticArgs& a) {
  PhaseScope ps(a.ctx, a.s, "init");
  hipLaunchKernelGGL(k_init, dim3(grid4(a.n)), dim3(kBlock), 0, a.s, a.n, a.n, a.P, a.count, vec_ok(a), a.ctx->dev,
                     (long long*)a.ncomp_user);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

cc_status static_run(StaticArgs& a) {
  cc_status st = a.o64 ? run_static<int64_t>(a, false) : run_static<int32_t>(a, false);
  record_stats_host(a);
  return st;
}

cc_status setup_args(StaticArgs& a, cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int o64,
                            const int32_t* adj, const cc_variant* v, void* ws, size_t ws_bytes, int32_t* labels,
                            int64_t* ncomp, void* stream) {
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  if (n < 1 || n > 0x7fffffffLL) return fail(CC_EINVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
  if (m < 0) return fail(CC_EINVAL, "m < 0");
  if (!o64 && m > 0x7fffffffLL) return fail(CC_EINVAL, "m=%lld needs 64-bit offsets", (long long)m);
  if (!offsets || !labels || (m > 0 && !adj)) return fail(CC_EINVAL, "NULL array argument");
  cc_status st = check_variant(v, false);
  if (st != CC_OK) return st;
  WsLayout L = ws_layout(n, m, v);
  if (!ws || ws_bytes < L.total)
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
  char* w = (char*)ws;
  a.ctx = ctx;
  a.s = (hipStream_t)stream;
  a.n = n;
  a.m = m;
  a.off = offsets;
  a.o64 = o64 != 0;
  a.adj = adj;
  a.v = v;
  a.L = L;
  a.ws = w;
  a.P = labels;
  a.count = (int32_t*)(w + L.count);
  a.cand = (int32_t*)(w + L.cand);
  a.big = (int32_t*)(w + L.big);
  a.heavy = (int32_t*)(w + L.heavy);
  a.hp = (long long*)(w + L.heavy + align256(heavy_cap(m) * 4));
  a.tsum = (long long*)(w + L.heavy + align256(heavy_cap(m) * 4) + align256((heavy_cap(m) + 1) * 8));
  a.hcap = (int64_t)heavy_cap(m);
  a.ncomp_user = ncomp;
  return CC_OK;
}

// Workspace of cc_connectivity_csr_noalloc: a fixed device array, one copy
// per device, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// device symbol): it takes the device address from hipGetSymbolAddress,
// once per device with that device current, when a context is created.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the caller has made the
// device current); looked up on the first request per device.
static cc_status noalloc_scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(CC_EDEVICE, "device %d beyond the %d supported", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(CC_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return CC_OK;
}

cc_status map_back_labels(StaticArgs& a, int64_t n, const int32_t* orig_of, const int32_t* new_of,
                          const int32_t* P, int32_t* labels_out) {
  PhaseScope ps(a.ctx, a.s, "mapback");
  const int64_t na = a.n;
  int32_t* rmin = a.map_rmin;
  // the compaction area is free once the labels are out
  int32_t* part = (int32_t*)(a.ws + a.L.seg);
  const unsigned g = grid_for((na + 3) / 4, kBlock, 2048);
  uint32_t* in_giant = (uint32_t*)(a.ws + a.L.bits);  // the bitmap area is free too
  const int aligned = (((uintptr_t)P | (uintptr_t)orig_of | (uintptr_t)new_of | (uintptr_t)labels_out) & 15u) == 0;
  hipLaunchKernelGGL(k_map_min, dim3(g), dim3(kBlock), 0, a.s, na, P, orig_of, rmin, (const DevScalars*)a.ctx->dev,
                     part, in_giant, aligned);
  if (a.o64)
    hipLaunchKernelGGL(k_map_giant<int64_t>, dim3(1), dim3(kBlock), 0, a.s, n, na, (const int64_t*)a.off, P,
                       a.ctx->dev, (const int32_t*)part, (int)g, rmin);
  else
    hipLaunchKernelGGL(k_map_giant<int32_t>, dim3(1), dim3(kBlock), 0, a.s, n, na, (const int32_t*)a.off, P,
                       a.ctx->dev, (const int32_t*)part, (int)g, rmin);
  hipLaunchKernelGGL(k_map_gather, dim3(grid_for((n + 3) / 4, kBlock, 4096)), dim3(kBlock), 0, a.s, n, P, new_of,
                     (const int32_t*)rmin, (const DevScalars*)a.ctx->dev, labels_out, aligned);
  hipLaunchKernelGGL(k_map_fix, dim3(grid_for((na + 31) / 32, kBlock, 4096)), dim3(kBlock), 0, a.s, n, P, orig_of,
                     (const int32_t*)rmin, (const DevScalars*)a.ctx->dev, (const uint32_t*)in_giant, labels_out);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

static void record_stats_host(StaticArgs& a) {
  cc_stats& s = a.ctx->last;
  s.n = a.n_parents > a.n ? a.n_parents : a.n;  // the graph's vertices, swept or not
  s.m = a.m;
  s.sample_success = a.sample_success;
  s.sample_rounds = a.sample_rounds;
  s.finish_rounds = a.finish_rounds;
}

}  // namespace cc

using namespace cc;

extern "C" {

cc_status cc_ctx_create(int device, cc_ctx** out) {
  if (!out) return fail(CC_EINVAL, "out is NULL");
  *out = nullptr;
  int cnt = 0;
  CC_HIP(hipGetDeviceCount(&cnt));
  if (device < 0 || device >= cnt) return fail(CC_EINVAL, "device %d not in [0, %d)", device, cnt);
  CC_HIP(hipSetDevice(device));
  cc_ctx* c = new cc_ctx();
  c->device = device;
  if (hipMalloc((void**)&c->dev, sizeof(DevScalars)) != hipSuccess ||
      hipHostMalloc((void**)&c->host, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&c->sel_host, 256, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
      hipHostGetDevicePointer((void**)&c->sel_dev, c->sel_host, 0) != hipSuccess ||
      hipHostMalloc((void**)&c->ring_host, 256, hipHostMallocDefault) != hipSuccess) {
    if (c->dev) (void)hipFree(c->dev);
    if (c->host) (void)hipHostFree(c->host);
    if (c->sel_host) (void)hipHostFree(c->sel_host);
    delete c;
    return fail(CC_ENOMEM, "cannot allocate context state");
  }
  if (hipEventCreateWithFlags(&c->ring_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ring_ev[1], hipEventDisableTiming) != hipSuccess) {
    cc_ctx_destroy(c);
    return fail(CC_EDEVICE, "cannot create the context's events");
  }
  CC_HIP(hipMemset(c->dev, 0, sizeof(DevScalars)));
  memset(c->host, 0, sizeof(DevScalars));
  CC_HIP(hipDeviceSynchronize());
  if (noalloc_scratch_address(device, &c->noalloc_scratch) != CC_OK) {
    const std::string msg = cc_last_error();
    cc_ctx_destroy(c);
    return fail(CC_EDEVICE, "%s", msg.c_str());
  }
  *out = c;
  return CC_OK;
}

void cc_ctx_destroy(cc_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& r : ctx->pending) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->dev) (void)hipFree(ctx->dev);
  if (ctx->host) (void)hipHostFree(ctx->host);
  if (ctx->sel_host) (void)hipHostFree(ctx->sel_host);
  if (ctx->ring_host) (void)hipHostFree(ctx->ring_host);
  for (hipEvent_t e : ctx->ring_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->amsf_host) (void)hipHostFree(ctx->amsf_host);
  delete ctx;
}

cc_status cc_ctx_sync_status(cc_ctx* ctx) {
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  CC_HIP(hipDeviceSynchronize());
  uint32_t err = 0;
  CC_HIP(hipMemcpy(&err, &ctx->dev->error, sizeof(err), hipMemcpyDeviceToHost));
  if (err) {
    uint32_t z = 0;
    CC_HIP(hipMemcpy(&ctx->dev->error, &z, sizeof(z), hipMemcpyHostToDevice));
    if (err & kErrRoundCap) return fail(CC_ELIVELOCK, "device error word 0x%x: round cap exceeded", err);
    return fail(CC_EDEVICE, "device error word 0x%x (1: id out of range, 4: malformed CSR)", err);
  }
  return CC_OK;
}

cc_status cc_last_stats(cc_ctx* ctx, cc_stats* out) {
  if (!ctx || !out) return fail(CC_EINVAL, "NULL argument");
  CC_HIP(hipDeviceSynchronize());
  CC_HIP(hipMemcpy(ctx->host, ctx->dev, sizeof(DevScalars), hipMemcpyDeviceToHost));
  cc_stats s = ctx->last;
  s.lmax = ctx->host->lmax;
  s.lmax_size = ctx->host->lmax_size;
  s.candidates = (int64_t)ctx->host->bin_count[0] + ctx->host->bin_count[1] + ctx->host->bin_count[2];
  s.candidate_edges = ctx->host->cand_edges;
  s.num_components = ctx->host->num_components;
  s.sample_bottom_up = ctx->host->bu_rounds;
  s.reserved = 0;
  *out = s;
  return CC_OK;
}

cc_status cc_ctx_set_round_limit(cc_ctx* ctx, int32_t limit) {
  if (!ctx || limit < 0) return fail(CC_EINVAL, "bad argument");
  ctx->round_limit = limit;
  return CC_OK;
}

cc_status cc_ctx_set_timing(cc_ctx* ctx, int enable) {
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  ctx->timing = enable;
  return CC_OK;
}

cc_status cc_ctx_set_timing_phase(cc_ctx* ctx, const char* name) {
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  ctx->timing_only = name ? name : "";
  return CC_OK;
}

int cc_phase_times(cc_ctx* ctx, int max_phases, const char** names, double* total_ms, int64_t* counts) {
  if (!ctx) return -1;
  harvest(ctx);
  int k = (int)ctx->phase_names.size();
  for (int i = 0; i < k && i < max_phases; ++i) {
    if (names) names[i] = ctx->phase_names[i].c_str();
    if (total_ms) total_ms[i] = ctx->phase_ms[i];
    if (counts) counts[i] = ctx->phase_cnt[i];
  }
  return k;
}

void cc_phase_times_reset(cc_ctx* ctx) {
  if (!ctx) return;
  harvest(ctx);
  for (auto& x : ctx->phase_ms) x = 0.0;
  for (auto& x : ctx->phase_cnt) x = 0;
}

cc_status cc_default_variant(cc_variant* out) {
  if (!out) return fail(CC_EINVAL, "out is NULL");
  memset(out, 0, sizeof(*out));
  out->sample = CC_SAMPLE_KOUT;
  out->kout_k = 2;
  out->kout_mode = CC_KOUT_HYBRID;
  out->bfs_tries = 3;
  out->ldd_beta = 0.2f;
  out->ldd_permute = 0;
  out->finish = CC_FIN_UF_REM_CAS;
  out->find = CC_FIND_NAIVE;
  out->splice = CC_SPLICE_SPLIT_ONE;
  out->lt_rules = CC_LT_PRF;
  out->seed = 0x5eed;
  return CC_OK;
}

cc_status cc_check_variant(const cc_variant* v) { return check_variant(v, false); }

cc_status cc_workspace_bytes(int64_t n, int64_t m, const cc_variant* v, size_t* bytes) {
  if (!bytes) return fail(CC_EINVAL, "bytes is NULL");
  if (n < 1 || n > 0x7fffffffLL || m < 0) return fail(CC_EINVAL, "bad n or m");
  cc_status st = check_variant(v, false);
  if (st != CC_OK) return st;
  *bytes = ws_layout(n, m, v).total;
  return CC_OK;
}

cc_status cc_connectivity_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                              const int32_t* adj, const cc_variant* v, void* workspace, size_t ws_bytes,
                              int32_t* labels_out, int64_t* num_components_dev, void* hip_stream) {
  StaticArgs a;
  cc_status st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, v, workspace, ws_bytes, labels_out,
                            num_components_dev, hip_stream);
  if (st != CC_OK) return st;
  st = a.o64 ? run_static<int64_t>(a, false) : run_static<int32_t>(a, false);
  record_stats_host(a);
  return st;
}

cc_status cc_mapped_workspace_bytes(int64_t n, int64_t m, const cc_variant* v, size_t* bytes) {
  size_t base = 0;
  cc_status st = cc_workspace_bytes(n, m, v, &base);
  if (st != CC_OK) return st;
  *bytes = base + align256((size_t)n * 4);  // the labels in the CSR's numbering
  return CC_OK;
}

cc_status cc_connectivity_csr_mapped(cc_ctx* ctx, int64_t n, int64_t n_active, int64_t m, const void* offsets,
                                     int offsets_are_64bit, const int32_t* adj, const int32_t* orig_of,
                                     const int32_t* new_of, const cc_variant* v, void* workspace, size_t ws_bytes,
                                     int32_t* labels_out, int64_t* num_components_dev, void* hip_stream) {
  if (!orig_of || !new_of) return fail(CC_EINVAL, "NULL permutation argument");
  if (n_active < 0 || n_active > n) return fail(CC_EINVAL, "n_active=%lld outside [0, n]", (long long)n_active);
  size_t base = 0;
  cc_status st = cc_workspace_bytes(n, m, v, &base);
  if (st != CC_OK) return st;
  if (!workspace || ws_bytes < base + align256((size_t)n * 4))
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                base + align256((size_t)n * 4));
  if (!labels_out) return fail(CC_EINVAL, "labels_out is NULL");
  // The algorithm runs on the first na vertices only: the others have no
  // edges, so each is a component of its own, labelled by the gather below
  // (one vertex at least, so that a graph without edges is a call too).
  const int64_t na = n_active > 0 ? n_active : 1;
  int32_t* Pnew = (int32_t*)((char*)workspace + base);
  StaticArgs a;
  st = setup_args(a, ctx, na, m, offsets, offsets_are_64bit, adj, v, workspace, base, Pnew, num_components_dev,
                  hip_stream);
  if (st != CC_OK) return st;
  a.n_parents = n;
  a.kout_by_xcd = false;
  // the count array is free once the finish has run: the output sweep
  // starts each root's minimum original id there
  a.map_orig = orig_of;
  a.map_rmin = a.count;
  st = a.o64 ? run_static<int64_t>(a, false) : run_static<int32_t>(a, false);
  if (st == CC_OK) st = map_back_labels(a, n, orig_of, new_of, Pnew, labels_out);
  record_stats_host(a);
  return st;
}

size_t cc_noalloc_scratch_bytes(void) { return kNoallocScratchBytes; }

cc_status cc_connectivity_csr_noalloc(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                                      const int32_t* adj, const cc_variant* v, int32_t* labels_out,
                                      int64_t* num_components_dev, void* hip_stream) {
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  if (!ctx->noalloc_scratch) return fail(CC_EDEVICE, "the context has no scratch array");
  size_t need = 0;
  cc_status st = cc_workspace_bytes(n, m, v, &need);
  if (st != CC_OK) return st;
  if (need > kNoallocScratchBytes)
    return fail(CC_ENOMEM, "n=%lld, m=%lld needs %zu bytes of workspace; the no-allocation entry point holds %zu",
                (long long)n, (long long)m, need, kNoallocScratchBytes);
  StaticArgs a;
  st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, v, ctx->noalloc_scratch, kNoallocScratchBytes,
                  labels_out, num_components_dev, hip_stream);
  if (st != CC_OK) return st;
  // phase events would create HIP events on first use: none in this call
  const int timing = ctx->timing;
  ctx->timing = 0;
  st = a.o64 ? run_static<int64_t>(a, false) : run_static<int32_t>(a, false);
  ctx->timing = timing;
  record_stats_host(a);
  return st;
}

cc_status cc_sample_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                        const int32_t* adj, const cc_variant* v, void* workspace, size_t ws_bytes,
                        int32_t* labels_out, int32_t* lmax_out_host, void* hip_stream) {
  StaticArgs a;
  cc_status st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, v, workspace, ws_bytes, labels_out,
                            nullptr, hip_stream);
  if (st != CC_OK) return st;
  st = a.o64 ? run_static<int64_t>(a, true) : run_static<int32_t>(a, true);
  record_stats_host(a);
  if (st != CC_OK) return st;
  int32_t lm = -1;
  CC_HIP(hipMemcpyAsync(&ctx->host->lmax, &ctx->dev->lmax, sizeof(int32_t), hipMemcpyDeviceToHost, a.s));
  CC_HIP(hipStreamSynchronize(a.s));
  lm = ctx->host->lmax;
  if (lmax_out_host) *lmax_out_host = lm;
  return CC_OK;
}

// Pair-list entry: a symmetric deduplicated CSR is built in the front of the
// workspace (offsets, adjacency, edge count), then the CSR path runs on the
// rest, which also serves as the build's scratch (the two never overlap in
// time on one stream).
struct CooLayout {
  int o64 = 0;
  size_t off = 0, adj = 0, mdev = 0, rest = 0, rest_bytes = 0, total = 0;
};

static cc_status coo_layout(int64_t n, int64_t num_pairs, const cc_variant* v, CooLayout* L) {
  if (n < 1 || n > 0x7fffffffLL || num_pairs < 0) return fail(CC_EINVAL, "bad n or num_pairs");
  cc_status st = check_variant(v, false);
  if (st != CC_OK) return st;
  size_t build = 0;
  st = cc_csr_workspace_bytes(n, num_pairs, &build);
  if (st != CC_OK) return st;
  const int64_t mmax = 2 * num_pairs;
  L->o64 = mmax > 0x7fffffffLL;
  size_t o = 0;
  L->off = o, o += align256((size_t)(n + 1) * (L->o64 ? 8 : 4));
  L->adj = o, o += align256((size_t)(mmax > 0 ? mmax : 1) * 4);
  L->mdev = o, o += 256;
  L->rest = o;
  L->rest_bytes = std::max(build, ws_layout(n, mmax, v).total);
  L->total = o + L->rest_bytes + 256;  // + alignment of the caller's base
  return CC_OK;
}

cc_status cc_coo_workspace_bytes(int64_t n, int64_t num_pairs, const cc_variant* v, size_t* bytes) {
  if (!bytes) return fail(CC_EINVAL, "bytes is NULL");
  CooLayout L;
  cc_status st = coo_layout(n, num_pairs, v, &L);
  if (st != CC_OK) return st;
  *bytes = L.total;
  return CC_OK;
}

cc_status cc_connectivity_coo(cc_ctx* ctx, int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v,
                              const cc_variant* var, void* workspace, size_t ws_bytes, int32_t* labels_out,
                              int64_t* num_components_dev, void* hip_stream) {
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  CooLayout L;
  cc_status st = coo_layout(n, num_pairs, var, &L);
  if (st != CC_OK) return st;
  if (!workspace || ws_bytes < L.total)
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, L.total);
  if (num_pairs > 0 && (!u || !v)) return fail(CC_EINVAL, "null pair arrays");
  char* w = (char*)(((uintptr_t)workspace + 255) & ~(uintptr_t)255);
  hipStream_t s = (hipStream_t)hip_stream;
  st = cc_build_csr(ctx, n, num_pairs, u, v, 1, w + L.rest, L.rest_bytes, w + L.off, L.o64, (int32_t*)(w + L.adj),
                    (int64_t*)(w + L.mdev), hip_stream);
  if (st != CC_OK) return st;
  int64_t m = 0;
  CC_HIP(hipMemcpyAsync(&m, w + L.mdev, sizeof(m), hipMemcpyDeviceToHost, s));
  CC_HIP(hipStreamSynchronize(s));
  return cc_connectivity_csr(ctx, n, m, w + L.off, L.o64, (const int32_t*)(w + L.adj), var, w + L.rest,
                             L.rest_bytes, labels_out, num_components_dev, hip_stream);
}

const char* cc_status_string(cc_status st) {
  switch (st) {
    case CC_OK: return "CC_OK";
    case CC_EINVAL: return "CC_EINVAL";
    case CC_ENOMEM: return "CC_ENOMEM";
    case CC_EDEVICE: return "CC_EDEVICE";
    case CC_ELIVELOCK: return "CC_ELIVELOCK";
    case CC_EBUSY: return "CC_EBUSY";
    case CC_EUNSUPPORTED: return "CC_EUNSUPPORTED";
  }
  return "CC_?";
}

const char* cc_last_error(void) { return g_err; }

}  // extern "C"
