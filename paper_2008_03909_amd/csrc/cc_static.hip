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
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "cc_device.h"
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
  if (ctx && ctx->timing) {
    a = get_event(ctx);
    if (a) hipEventRecord(a, s);
  }
}

PhaseScope::~PhaseScope() {
  if (!a) return;
  hipEvent_t b = get_event(ctx);
  if (!b) return;
  hipEventRecord(b, s);
  ctx->pending.push_back({name, a, b});
}

static void harvest(cc_ctx* ctx) {
  for (auto& r : ctx->pending) {
    hipEventSynchronize(r.b);
    float ms = 0.f;
    hipEventElapsedTime(&ms, r.a, r.b);
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
    if (v->kout_mode < CC_KOUT_HYBRID || v->kout_mode > CC_KOUT_PURE) return fail(CC_EINVAL, "bad kout_mode");
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
      if (v->find < CC_FIND_NAIVE || v->find > CC_FIND_COMPRESS) return fail(CC_EINVAL, "bad find");
      break;
    case CC_FIN_SV:
      if (for_stream) return fail(CC_EUNSUPPORTED, "streams use union-find finishes");
      break;
    case CC_FIN_LT: {
      if (for_stream) return fail(CC_EUNSUPPORTED, "streams use union-find finishes");
      uint32_t r = v->lt_rules;
      const uint32_t ok[] = {CC_LT_CRSA, CC_LT_PRSA, CC_LT_PRS, CC_LT_CRFA, CC_LT_PRFA, CC_LT_PRF};
      bool found = false;
      for (uint32_t x : ok) found |= (r == x);
      if (!found) return fail(CC_EUNSUPPORTED, "only the root-based Liu-Tarjan variants are built (rules=%u)", r);
      break;
    }
    default:
      return fail(CC_EINVAL, "bad finish %d", v->finish);
  }
  return CC_OK;
}

WsLayout ws_layout(int64_t n, int64_t m, const cc_variant* v) {
  WsLayout L;
  size_t off = 0;
  const size_t n4 = align256((size_t)n * 4);
  L.count = off, off += n4;
  L.cand = off, off += n4;
  L.big = off, off += n4;
  if (v->sample == CC_SAMPLE_BFS || v->sample == CC_SAMPLE_LDD) {
    L.bits = off, off += 3 * align256((size_t)((n + 31) / 32) * 4);
    L.queue = off, off += 2 * n4;
  }
  if (v->sample == CC_SAMPLE_LDD) L.hist = off, off += align256(4096 * 4);
  if (v->finish == CC_FIN_LT && (v->lt_rules & CC_LT_ALTER)) L.edges = off, off += 2 * align256((size_t)m * 4);
  L.total = off + 256;
  return L;
}

// ---------------------------------------------------------------------------
// kernels
constexpr int kBlock = 256;
constexpr int64_t kStreamGridCap = 4096;

__global__ void k_init(int64_t n, int32_t* __restrict__ P, int32_t* __restrict__ count, DevScalars* sc,
                       long long* ncomp_user) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (i == 0) {
    sc->changed = 0;
    sc->lmax_key = 0ull;
    sc->lmax = -1;
    sc->bfs_min = 0x7fffffff;
    for (int b = 0; b < 4; ++b) sc->bin_count[b] = 0;
    sc->cand_edges = 0;
    sc->num_components = 0;
    sc->lmax_size = 0;
    sc->qcount[0] = sc->qcount[1] = 0;
    sc->frontier_edges = 0;
    sc->reached = 0;
    sc->flag2 = 0;
    if (ncomp_user) *ncomp_user = 0;
  }
  for (; i < n; i += stride) {
    P[i] = (int32_t)i;
    if (count) count[i] = 0;
  }
}

template <typename I>
__global__ void k_kout(int64_t n, const I* __restrict__ off, const int32_t* __restrict__ adj, int32_t* P, int k,
                       int mode, uint64_t key) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const int64_t b = (int64_t)off[v];
    const int64_t deg = (int64_t)off[v + 1] - b;
    if (deg <= 0) continue;
    for (int j = 0; j < k; ++j) {
      int64_t idx;
      if (mode == CC_KOUT_AFFOREST) {
        if (j >= deg) break;
        idx = j;
      } else if (mode == CC_KOUT_HYBRID && j == 0) {
        idx = 0;
      } else {
        idx = (int64_t)(sm_out(key, (uint64_t)v * (uint64_t)k + (uint64_t)j) % (uint64_t)deg);
      }
      union_rem<kSplitOne, kFindNaive>(P, (int32_t)v, adj[b + idx]);
    }
  }
}

// Full compression fused with the IdentifyFrequent histogram.  Only vertices
// with at least one edge are counted (an isolated vertex is its own class and
// can never be the most frequent one unless every class is a singleton, in
// which case skipping nothing is equivalent).  Equal labels inside a wave are
// aggregated into one atomic.
template <typename I>
__global__ void k_compress_count(int64_t n, const I* __restrict__ off, int32_t* P, int32_t* __restrict__ count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = lane_id();
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    const bool act = v < n;
    int32_t r = 0;
    bool c = false;
    if (act) {
      int32_t p = ld(P + v);
      r = p;
      if (p != (int32_t)v) {
        r = find_naive(P, p);
        if (r != p) st(P + v, r);
      }
      c = (int64_t)off[v + 1] > (int64_t)off[v];
    }
    if (!count) continue;
    uint64_t mact = __ballot(c);
    if (mact == 0) continue;
    const int leader = __ffsll((unsigned long long)mact) - 1;
    const int32_t lead = __shfl(r, leader, kWave);
    const uint64_t same = __ballot(c && r == lead);
    if (c) {
      if (r == lead) {
        if (lane == leader)
          __hip_atomic_fetch_add(count + lead, (int32_t)__popcll(same), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        __hip_atomic_fetch_add(count + r, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
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

// IdentifyFrequent: max over (count << 32 | ~label); ties go to the smaller label.
__global__ void k_argmax(int64_t n, const int32_t* __restrict__ count, DevScalars* sc) {
  __shared__ unsigned long long red[kBlock / kWave];
  unsigned long long best = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    int32_t c = count[v];
    if (c > 0) {
      unsigned long long key = ((unsigned long long)(uint32_t)c << 32) | (uint32_t)(~(uint32_t)v);
      best = key > best ? key : best;
    }
  }
  best = wave_max_u64(best);
  if (lane_id() == 0) red[threadIdx.x / kWave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) best = red[w] > best ? red[w] : best;
    if (best) atomicMax(&sc->lmax_key, best);
  }
}

__device__ __forceinline__ int32_t lmax_of(unsigned long long key) {
  return key ? (int32_t)(~(uint32_t)(key & 0xffffffffull)) : -1;
}

__global__ void k_resolve_lmax(DevScalars* sc, int use) {
  unsigned long long key = sc->lmax_key;
  sc->lmax = use ? lmax_of(key) : -1;
  sc->lmax_size = use ? (long long)(key >> 32) : 0;
}

// Candidate compaction with degree binning.
template <typename I>
__global__ void k_compact(int64_t n, const I* __restrict__ off, const int32_t* __restrict__ P, DevScalars* sc,
                          int32_t* __restrict__ cand, int32_t* __restrict__ big, int thr_wave, int thr_block) {
  const int32_t L = sc->lmax;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = lane_id();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  long long edges = 0;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    int64_t deg = 0;
    bool isc = false;
    if (v < n) {
      deg = (int64_t)off[v + 1] - (int64_t)off[v];
      isc = deg > 0 && P[v] != L;
    }
    const int bin = deg <= thr_wave ? 0 : (deg <= thr_block ? 1 : 2);
    if (isc) edges += deg;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const uint64_t mask = __ballot(isc && bin == b);
      if (!mask) continue;
      const int leader = __ffsll((unsigned long long)mask) - 1;
      int32_t basepos = 0;
      if (lane == leader)
        basepos = __hip_atomic_fetch_add(&sc->bin_count[b], (int32_t)__popcll(mask), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
      basepos = __shfl(basepos, leader, kWave);
      if (isc && bin == b) {
        const int32_t pos = basepos + (int32_t)__popcll(mask & lt_mask);
        if (b == 0) cand[pos] = (int32_t)v;
        else if (b == 1) big[pos] = (int32_t)v;
        else big[n - 1 - pos] = (int32_t)v;
      }
    }
  }
  edges = wave_sum(edges);
  if (lane == 0 && edges) add64(&sc->cand_edges, edges);
}

// Union-find finish: thread / wave / block per candidate.
template <int ALG, int SPLICE, int FIND, typename I>
__global__ void k_fin_thread(const int32_t* __restrict__ cand, const DevScalars* sc, const I* __restrict__ off,
                             const int32_t* __restrict__ adj, int32_t* P) {
  const int64_t cnt = sc->bin_count[0];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt; i += stride) {
    const int32_t u = cand[i];
    const int64_t e = (int64_t)off[u + 1];
    for (int64_t j = (int64_t)off[u]; j < e; ++j) unite<ALG, SPLICE, FIND>(P, u, adj[j]);
  }
}

template <int ALG, int SPLICE, int FIND, typename I>
__global__ void k_fin_wave(const int32_t* __restrict__ big, const DevScalars* sc, const I* __restrict__ off,
                           const int32_t* __restrict__ adj, int32_t* P) {
  const int64_t cnt = sc->bin_count[1];
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
  const int lane = lane_id();
  for (int64_t i = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; i < cnt; i += waves) {
    const int32_t u = big[i];
    const int64_t e = (int64_t)off[u + 1];
    for (int64_t j = (int64_t)off[u] + lane; j < e; j += kWave) unite<ALG, SPLICE, FIND>(P, u, adj[j]);
  }
}

template <int ALG, int SPLICE, int FIND, typename I>
__global__ void k_fin_block(int64_t n, const int32_t* __restrict__ big, const DevScalars* sc,
                            const I* __restrict__ off, const int32_t* __restrict__ adj, int32_t* P) {
  const int64_t cnt = sc->bin_count[2];
  for (int64_t i = blockIdx.x; i < cnt; i += gridDim.x) {
    const int32_t u = big[n - 1 - i];
    const int64_t e = (int64_t)off[u + 1];
    for (int64_t j = (int64_t)off[u] + threadIdx.x; j < e; j += blockDim.x) unite<ALG, SPLICE, FIND>(P, u, adj[j]);
  }
}

// Final compression and component count: label = root (the component's
// minimum, since every link points to a smaller id).
__global__ void k_output(int64_t n, int32_t* P, DevScalars* sc, long long* ncomp_user) {
  __shared__ long long red[kBlock / kWave];
  long long roots = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const int32_t p = ld(P + v);
    if (p == (int32_t)v) {
      ++roots;
      continue;
    }
    const int32_t r = find_naive(P, p);
    if (r != p) st(P + v, r);
  }
  roots = wave_sum(roots);
  if (lane_id() == 0) red[threadIdx.x / kWave] = roots;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / kWave; ++w) roots += red[w];
    if (roots) {
      add64(&sc->num_components, roots);
      if (ncomp_user) add64(ncomp_user, roots);
    }
  }
}

// ---------------------------------------------------------------------------
// host orchestration

constexpr int kThrWave = 32;     // degree <= 32: one thread per candidate
constexpr int kThrBlock = 8192;  // degree <= 8192: one wave; larger: one block

template <int ALG, int SPLICE, int FIND, typename I>
static cc_status launch_uf_finish(StaticArgs& a) {
  const I* off = (const I*)a.off;
  const unsigned gt = grid_for(a.n, kBlock, kStreamGridCap);
  hipLaunchKernelGGL((k_fin_thread<ALG, SPLICE, FIND, I>), dim3(gt), dim3(kBlock), 0, a.s, a.cand, a.ctx->dev, off,
                     a.adj, a.P);
  const unsigned gw = grid_for(a.n * kWave, kBlock, 2048);
  hipLaunchKernelGGL((k_fin_wave<ALG, SPLICE, FIND, I>), dim3(gw), dim3(kBlock), 0, a.s, a.big, a.ctx->dev, off,
                     a.adj, a.P);
  hipLaunchKernelGGL((k_fin_block<ALG, SPLICE, FIND, I>), dim3(1024), dim3(kBlock), 0, a.s, a.n, a.big, a.ctx->dev,
                     off, a.adj, a.P);
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
    if (v->find == 0) return launch_uf_finish<1, 0, 0, I>(a);
    if (v->find == 1) return launch_uf_finish<1, 0, 1, I>(a);
    if (v->find == 2) return launch_uf_finish<1, 0, 2, I>(a);
    if (v->find == 3) return launch_uf_finish<1, 0, 3, I>(a);
  }
  return fail(CC_EINVAL, "no such union-find variant");
}

template <typename I>
cc_status compress_count_frequent(StaticArgs& a, bool use_lmax) {
  const unsigned g = grid_for(a.n, kBlock, kStreamGridCap);
  {
    PhaseScope ps(a.ctx, a.s, "compress_count");
    hipLaunchKernelGGL(k_compress_count<I>, dim3(g), dim3(kBlock), 0, a.s, a.n, (const I*)a.off, a.P,
                       use_lmax ? a.count : (int32_t*)nullptr);
  }
  {
    PhaseScope ps(a.ctx, a.s, "frequent");
    if (use_lmax) hipLaunchKernelGGL(k_argmax, dim3(g), dim3(kBlock), 0, a.s, a.n, (const int32_t*)a.count, a.ctx->dev);
    hipLaunchKernelGGL(k_resolve_lmax, dim3(1), dim3(1), 0, a.s, a.ctx->dev, use_lmax ? 1 : 0);
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
      hipLaunchKernelGGL(k_kout<I>, dim3(grid_for(a.n, kBlock, kStreamGridCap)), dim3(kBlock), 0, a.s, a.n,
                         (const I*)a.off, a.adj, a.P, v->kout_k, v->kout_mode, key);
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
static cc_status run_static(StaticArgs& a, bool sample_only) {
  {
    PhaseScope ps(a.ctx, a.s, "init");
    hipLaunchKernelGGL(k_init, dim3(grid_for(a.n, kBlock, kStreamGridCap)), dim3(kBlock), 0, a.s, a.n, a.P,
                       a.v->sample == CC_SAMPLE_NONE ? (int32_t*)nullptr : a.count, a.ctx->dev,
                       (long long*)a.ncomp_user);
    CC_LAUNCH_CHECK();
  }
  cc_status st = run_sample<I>(a);
  if (st != CC_OK || sample_only) return st;
  {
    PhaseScope ps(a.ctx, a.s, "compact");
    hipLaunchKernelGGL(k_compact<I>, dim3(grid_for(a.n, kBlock, kStreamGridCap)), dim3(kBlock), 0, a.s, a.n,
                       (const I*)a.off, (const int32_t*)a.P, a.ctx->dev, a.cand, a.big, kThrWave, kThrBlock);
    CC_LAUNCH_CHECK();
  }
  a.finish_rounds = 0;
  {
    PhaseScope ps(a.ctx, a.s, "finish");
    if (a.v->finish == CC_FIN_SV) st = finish_sv<I>(a);
    else if (a.v->finish == CC_FIN_LT) st = finish_lt<I>(a);
    else st = uf_finish_dispatch<I>(a);
  }
  if (st != CC_OK) return st;
  {
    PhaseScope ps(a.ctx, a.s, "output");
    hipLaunchKernelGGL(k_output, dim3(grid_for(a.n, kBlock, kStreamGridCap)), dim3(kBlock), 0, a.s, a.n, a.P,
                       a.ctx->dev, (long long*)a.ncomp_user);
    CC_LAUNCH_CHECK();
  }
  return CC_OK;
}

static cc_status setup_args(StaticArgs& a, cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int o64,
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
  a.ncomp_user = ncomp;
  return CC_OK;
}

static void record_stats_host(StaticArgs& a) {
  cc_stats& s = a.ctx->last;
  s.n = a.n;
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
      hipHostMalloc((void**)&c->host, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) {
    if (c->dev) hipFree(c->dev);
    delete c;
    return fail(CC_ENOMEM, "cannot allocate context state");
  }
  CC_HIP(hipMemset(c->dev, 0, sizeof(DevScalars)));
  memset(c->host, 0, sizeof(DevScalars));
  CC_HIP(hipDeviceSynchronize());
  *out = c;
  return CC_OK;
}

void cc_ctx_destroy(cc_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipDeviceSynchronize();
  for (auto& r : ctx->pending) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (auto e : ctx->event_pool) hipEventDestroy(e);
  if (ctx->dev) hipFree(ctx->dev);
  if (ctx->host) hipHostFree(ctx->host);
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
  *out = s;
  return CC_OK;
}

cc_status cc_ctx_set_timing(cc_ctx* ctx, int enable) {
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  ctx->timing = enable;
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
