// Spanning forest (ConnectIt appendix "ConnectIt: Spanning Forest"): the
// static algorithm with every sampled and finishing link recorded as an
// edge, then a filter of the recorded edges.
//
// Each forest edge is stored at a vertex slot that no other edge can take.
// BFS and LDD tree edges go to the child they claimed (tree_e); an edge
// that hooked a union-find root (k-out sampling, and the finish) goes to
// that root (hook_e).  The paper keeps one array; two are kept here because
// this library relabels every BFS/LDD cluster to its minimum member, which
// can be a claimed child and later a hooked root.  Each slot is written at
// most once, there are n - c recorded edges in all, and they span every
// component without a cycle.  Only root-based finishes that hook with a CAS
// are supported: UF-Async, UF-Early, UF-Hooks, and UF-Rem-CAS with
// SplitAtomicOne or HalveAtomicOne (those only shorten paths inside a tree).  SpliceAtomic
// re-parents a non-root into the other tree, a link no recorded edge
// stands for; SV and LT hook with writeMin, which does not identify the
// winning edge, and label propagation keeps no tree at all.
#include "cc_static.h"

namespace cc {

constexpr int kForestTile = 4096;   // entries of the (tree_e ++ hook_e) array per block

// Slot i of the concatenation (tree_e ++ hook_e), or of hook_e alone when
// there is no tree array.
__device__ __forceinline__ int2 forest_slot(const int2* tree, const int2* hook, int64_t n, int64_t i) {
  if (!tree) return hook[i];
  return i < n ? tree[i] : hook[i - n];
}

__global__ void __launch_bounds__(kFBlock) k_forest_count(int64_t len, const int2* __restrict__ tree,
                                                          const int2* __restrict__ hook, int64_t n,
                                                          int32_t* __restrict__ cnt) {
  __shared__ int32_t red[kFBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kForestTile;
  int32_t c = 0;
  for (int64_t i = base + threadIdx.x; i < base + kForestTile && i < len; i += kFBlock) {
    const int2 e = forest_slot(tree, hook, n, i);
    c += e.x >= 0;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
  if (lane_id() == 0) red[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t s = 0;
    for (int w = 0; w < kFBlock / kWave; ++w) s += red[w];
    cnt[blockIdx.x] = s;
  }
}

// One block: exclusive scan of the per-tile counts, total to *total.
__global__ void __launch_bounds__(1024) k_forest_scan(int64_t tiles, int32_t* cnt, long long* total) {
  __shared__ long long wsum[1024 / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  long long carry = 0;
  for (int64_t b = 0; b < tiles; b += 1024) {
    const int64_t i = b + threadIdx.x;
    const long long x = i < tiles ? cnt[i] : 0;
    long long inc = x;
    for (int o = 1; o < kWave; o <<= 1) {
      const long long y = __shfl_up(inc, o, kWave);
      if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    long long before = 0, all = 0;
    for (int q = 0; q < 1024 / kWave; ++q) {
      if (q < w) before += wsum[q];
      all += wsum[q];
    }
    if (i < tiles) cnt[i] = (int32_t)(carry + before + inc - x);
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(kFBlock) k_forest_write(int64_t len, const int2* __restrict__ tree,
                                                          const int2* __restrict__ hook,
                                                          const float* __restrict__ hook_w, int64_t n,
                                                          const int32_t* __restrict__ base_of,
                                                          int32_t* __restrict__ out_u, int32_t* __restrict__ out_v,
                                                          float* __restrict__ out_w,
                                                          const int32_t* __restrict__ orig_of) {
  __shared__ int32_t wcnt[kFBlock / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kForestTile;
  int32_t pos = base_of[blockIdx.x];
  for (int64_t i0 = base; i0 < base + kForestTile && i0 < len; i0 += kFBlock) {
    const int64_t i = i0 + threadIdx.x;
    int2 e = make_int2(-1, -1);
    if (i < base + kForestTile && i < len) e = forest_slot(tree, hook, n, i);
    const bool keep = e.x >= 0;
    const uint64_t m = __ballot(keep);
    if (lane == 0) wcnt[w] = __popcll(m);
    __syncthreads();
    int32_t before = 0, all = 0;
    for (int q = 0; q < kFBlock / kWave; ++q) {
      if (q < w) before += wcnt[q];
      all += wcnt[q];
    }
    if (keep) {
      const int32_t p = pos + before + __popcll(m & lt);
      out_u[p] = orig_of ? orig_of[e.x] : e.x;
      out_v[p] = orig_of ? orig_of[e.y] : e.y;
      if (out_w) out_w[p] = hook_w[tree ? i - n : i];
    }
    pos += all;
    __syncthreads();
  }
}

int64_t forest_tiles(int64_t len) { return (len + kForestTile - 1) / kForestTile; }

cc_status forest_filter(hipStream_t s, int64_t n, const int2* tree, const int2* hook, const float* hook_w,
                        int32_t* cnt, int32_t* out_u, int32_t* out_v, float* out_w, int64_t* num_edges,
                        const int32_t* orig_of) {
  const int64_t len = tree ? 2 * n : n;
  const int64_t tiles = forest_tiles(len);
  hipLaunchKernelGGL(k_forest_count, dim3((unsigned)tiles), dim3(kFBlock), 0, s, len, tree, hook, n, cnt);
  hipLaunchKernelGGL(k_forest_scan, dim3(1), dim3(1024), 0, s, tiles, cnt, (long long*)num_edges);
  hipLaunchKernelGGL(k_forest_write, dim3((unsigned)tiles), dim3(kFBlock), 0, s, len, tree, hook,
                     (hook_w && out_w) ? hook_w : (const float*)nullptr, n, (const int32_t*)cnt, out_u, out_v,
                     (hook_w && out_w) ? out_w : (float*)nullptr, orig_of);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

static size_t forest_extra(int64_t n) {
  return 2 * align256((size_t)n * 8) + align256((size_t)forest_tiles(2 * n) * 4);
}

}  // namespace cc

using namespace cc;

extern "C" {

cc_status cc_forest_workspace_bytes(int64_t n, int64_t m, const cc_variant* v, size_t* bytes) {
  if (!bytes) return fail(CC_EINVAL, "bytes is NULL");
  size_t base = 0;
  cc_status st = cc_workspace_bytes(n, m, v, &base);
  if (st != CC_OK) return st;
  *bytes = align256(base) + forest_extra(n);
  return CC_OK;
}

cc_status cc_spanning_forest_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                                 const int32_t* adj, const cc_variant* v, void* workspace, size_t ws_bytes,
                                 int32_t* labels_out, int32_t* edges_u, int32_t* edges_v, int64_t* num_edges_dev,
                                 void* hip_stream) {
  if (!v) return fail(CC_EINVAL, "variant is NULL");
  if (v->finish != CC_FIN_UF_REM_CAS && v->finish != CC_FIN_UF_ASYNC && v->finish != CC_FIN_UF_EARLY &&
      v->finish != CC_FIN_UF_HOOKS)
    return fail(CC_EUNSUPPORTED, "spanning forest needs a union-find finish (Rem-CAS, Async, Early or Hooks)");
  if (v->finish == CC_FIN_UF_REM_CAS && v->splice == CC_SPLICE_ATOMIC)
    return fail(CC_EUNSUPPORTED, "spanning forest: SpliceAtomic moves non-roots between trees without a hook");
  if (!edges_u || !edges_v || !num_edges_dev) return fail(CC_EINVAL, "NULL forest output");
  size_t need = 0;
  cc_status st = cc_forest_workspace_bytes(n, m, v, &need);
  if (st != CC_OK) return st;
  if (!workspace || ws_bytes < need)
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
  size_t base = 0;
  cc_workspace_bytes(n, m, v, &base);
  base = align256(base);
  StaticArgs a;
  st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, v, workspace, base, labels_out, nullptr, hip_stream);
  if (st != CC_OK) return st;
  char* w = (char*)workspace + base;
  a.tree_e = (int2*)w;
  a.hook_e = (int2*)(w + align256((size_t)n * 8));
  int32_t* cnt = (int32_t*)(w + 2 * align256((size_t)n * 8));
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(4 * n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, (uint32_t*)a.tree_e,
                     2 * n, 0xffffffffu);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(4 * n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, (uint32_t*)a.hook_e,
                     2 * n, 0xffffffffu);
  CC_LAUNCH_CHECK();
  st = static_run(a);
  if (st != CC_OK) return st;
  return forest_filter(a.s, n, a.tree_e, a.hook_e, nullptr, cnt, edges_u, edges_v, nullptr, num_edges_dev);
}

cc_status cc_forest_mapped_workspace_bytes(int64_t n, int64_t m, const cc_variant* v, size_t* bytes) {
  if (!bytes) return fail(CC_EINVAL, "bytes is NULL");
  size_t f = 0;
  cc_status st = cc_forest_workspace_bytes(n, m, v, &f);
  if (st != CC_OK) return st;
  *bytes = f + align256((size_t)n * 4);  // the labels in the CSR's numbering
  return CC_OK;
}

cc_status cc_spanning_forest_csr_mapped(cc_ctx* ctx, int64_t n, int64_t n_active, int64_t m, const void* offsets,
                                        int offsets_are_64bit, const int32_t* adj, const int32_t* orig_of,
                                        const int32_t* new_of, const cc_variant* v, void* workspace, size_t ws_bytes,
                                        int32_t* labels_out, int32_t* edges_u, int32_t* edges_v,
                                        int64_t* num_edges_dev, void* hip_stream) {
  if (!v) return fail(CC_EINVAL, "variant is NULL");
  if (v->finish != CC_FIN_UF_REM_CAS && v->finish != CC_FIN_UF_ASYNC && v->finish != CC_FIN_UF_EARLY &&
      v->finish != CC_FIN_UF_HOOKS)
    return fail(CC_EUNSUPPORTED, "spanning forest needs a union-find finish (Rem-CAS, Async, Early or Hooks)");
  if (v->finish == CC_FIN_UF_REM_CAS && v->splice == CC_SPLICE_ATOMIC)
    return fail(CC_EUNSUPPORTED, "spanning forest: SpliceAtomic moves non-roots between trees without a hook");
  if (!edges_u || !edges_v || !num_edges_dev || !labels_out) return fail(CC_EINVAL, "NULL output");
  if (!orig_of || !new_of) return fail(CC_EINVAL, "NULL permutation argument");
  if (n_active < 0 || n_active > n) return fail(CC_EINVAL, "n_active=%lld outside [0, n]", (long long)n_active);
  size_t need = 0;
  cc_status st = cc_forest_mapped_workspace_bytes(n, m, v, &need);
  if (st != CC_OK) return st;
  if (!workspace || ws_bytes < need)
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
  size_t base = 0;
  cc_workspace_bytes(n, m, v, &base);
  base = align256(base);
  // as cc_connectivity_csr_mapped: the algorithm on the first na vertices,
  // the others (empty rows) alone in their components and without edges
  const int64_t na = n_active > 0 ? n_active : 1;
  char* w = (char*)workspace + base;
  int32_t* Pnew = (int32_t*)(w + forest_extra(n));
  StaticArgs a;
  st = setup_args(a, ctx, na, m, offsets, offsets_are_64bit, adj, v, workspace, base, Pnew, nullptr, hip_stream);
  if (st != CC_OK) return st;
  a.n_parents = n;
  a.kout_by_xcd = false;
  a.map_orig = orig_of;
  a.map_rmin = a.count;
  // slot arrays sized for all n vertices (a hook or claim beyond na, which
  // only a broken n_active makes, lands in a slot the filter never reads);
  // the filter reads the first na of each
  a.tree_e = (int2*)w;
  a.hook_e = (int2*)(w + align256((size_t)n * 8));
  int32_t* cnt = (int32_t*)(w + 2 * align256((size_t)n * 8));
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(4 * na, kFBlock, 4096)), dim3(kFBlock), 0, a.s, (uint32_t*)a.tree_e,
                     2 * na, 0xffffffffu);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(4 * na, kFBlock, 4096)), dim3(kFBlock), 0, a.s, (uint32_t*)a.hook_e,
                     2 * na, 0xffffffffu);
  CC_LAUNCH_CHECK();
  st = static_run(a);
  if (st != CC_OK) return st;
  st = forest_filter(a.s, na, a.tree_e, a.hook_e, nullptr, cnt, edges_u, edges_v, nullptr, num_edges_dev, orig_of);
  if (st != CC_OK) return st;
  return map_back_labels(a, n, orig_of, new_of, Pnew, labels_out);
}

}  // extern "C"
