// Ingest: undirected pair list -> symmetric CSR on the device.
//
// The CSR format is the one of ConnectIt Section 2 ("Graph Notation and
// Formats"): offsets I with I[n] = m and the neighbours of v in
// A[I[v]] .. A[I[v+1]-1].  Rows are sorted ascending, so the k-out sampler's
// "first edge" is the smallest neighbour.
//
//   expand   every pair (u, v), u != v, emits the 64-bit keys (u<<32 | v) and
//            (v<<32 | u); ids outside [0, n) set the error word and drop out
//   sort     stable LSD radix sort on the low ceil(log2 n) bits of both
//            halves (8-bit digits): per-tile digit histograms, one exclusive
//            scan over the digit-major histogram table, stable scatter with
//            in-tile ranks from wave ballots
//   dedup    optional: keep a key iff it differs from its predecessor
//   emit     A[i] = low half; I[v] = first i whose high half is >= v
#include <vector>

#include "cc_frontier.h"
#include "cc_static.h"

namespace cc {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per block
constexpr int kWavesPerSortBlock = kSortThreads / kWave;

// Pair i writes keys 2i and 2i+1; a self-loop or a pair with an id outside
// [0, n) writes two sentinel keys (all ones), which sort after every real key
// because a real key never has all-ones digits in both halves (that would be
// the self-loop (2^bits-1, 2^bits-1)).  The number of real keys is counted
// with one atomic per block.
constexpr unsigned long long kSentinel = ~0ull;

__global__ void __launch_bounds__(256) k_expand_pairs(int64_t n, int64_t num_pairs, const int32_t* __restrict__ u,
                                                      const int32_t* __restrict__ v,
                                                      unsigned long long* __restrict__ keys, unsigned long long* cnt,
                                                      DevScalars* sc) {
  __shared__ unsigned long long red[256 / kWave];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  unsigned long long real = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < num_pairs; i += stride) {
    const int32_t x = u[i], y = v[i];
    const bool ok = x >= 0 && y >= 0 && (int64_t)x < n && (int64_t)y < n;
    bad |= !ok;
    const bool take = ok && x != y;
    ulonglong2 kv;
    kv.x = take ? (((unsigned long long)(uint32_t)x << 32) | (uint32_t)y) : kSentinel;
    kv.y = take ? (((unsigned long long)(uint32_t)y << 32) | (uint32_t)x) : kSentinel;
    *(ulonglong2*)(keys + 2 * i) = kv;
    real += take ? 2ull : 0ull;
  }
  real = wave_sum(real);
  if (lane_id() == 0) red[threadIdx.x / kWave] = real;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 256 / kWave; ++w) real += red[w];
    if (real) __hip_atomic_fetch_add(cnt, real, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (__ballot(bad) && lane_id() == 0) atomicOr(&sc->error, kErrBadId);
}

__device__ __forceinline__ uint32_t digit_of(unsigned long long k, int shift, uint32_t mask) {
  return (uint32_t)(k >> shift) & mask;
}

// Per-tile digit histogram, stored digit-major: hist[d * nblocks + block].
__global__ void k_radix_hist(const unsigned long long* __restrict__ keys, int64_t count, int shift, uint32_t dmask,
                             uint32_t* __restrict__ hist, int64_t nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  for (int j = 0; j < kSortItems; ++j) {
    const int64_t i = base + (int64_t)j * kSortThreads + threadIdx.x;
    if (i < count) atomicAdd(&h[digit_of(keys[i], shift, dmask)], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter.  Within a tile the key order is (item j, thread t); ranks
// are assigned in that order.
__global__ void k_radix_scatter(const unsigned long long* __restrict__ keys, unsigned long long* __restrict__ out,
                                int64_t count, int shift, uint32_t dmask, const uint32_t* __restrict__ hist_scan,
                                int64_t nblocks) {
  __shared__ uint32_t gofs[256];
  __shared__ uint32_t wcnt[kWavesPerSortBlock][256];
  const int t = threadIdx.x;
  const int w = t / kWave;
  gofs[t] = hist_scan[(int64_t)t * nblocks + blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint64_t lt = lanemask_lt();
  for (int j = 0; j < kSortItems; ++j) {
    for (int q = 0; q < kWavesPerSortBlock; ++q) wcnt[q][t] = 0;
    __syncthreads();
    const int64_t i = base + (int64_t)j * kSortThreads + t;
    const bool valid = i < count;
    unsigned long long k = 0;
    uint32_t d = 0;
    if (valid) {
      k = keys[i];
      d = digit_of(k, shift, dmask);
    }
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t mb = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? mb : ~mb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    // exclusive prefix over waves for digit t, then advance the tile offset
    {
      uint32_t run = gofs[t];
      for (int q = 0; q < kWavesPerSortBlock; ++q) {
        const uint32_t c = wcnt[q][t];
        wcnt[q][t] = run;
        run += c;
      }
      gofs[t] = run;
    }
    __syncthreads();
    if (valid) out[(int64_t)wcnt[w][d] + rank] = k;
    __syncthreads();
  }
}

// ---- device-wide exclusive scan of uint32 (in place) ----------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t ws[kScanThreads / kWave];
  const int lane = lane_id(), w = threadIdx.x / kWave;
  uint32_t inc = x;
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) ws[w] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (int q = 0; q < kScanThreads / kWave; ++q) {
    if (q < w) before += ws[q];
    all += ws[q];
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

__global__ void k_scan_reduce(const uint32_t* __restrict__ a, int64_t count, uint32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t s = 0;
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < count) s += a[base + j];
  uint32_t total;
  block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Single block: exclusive scan of the tile sums.
__global__ void k_scan_top(uint32_t* sums, int64_t count) {
  uint32_t carry = 0;
  for (int64_t base = 0; base < count; base += kScanTile) {
    const int64_t b = base + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    for (int j = 0; j < kScanItems; ++j) {
      v[j] = (b + j < count) ? sums[b + j] : 0u;
      s += v[j];
    }
    uint32_t total;
    uint32_t ex = block_exclusive_scan(s, &total) + carry;
    for (int j = 0; j < kScanItems; ++j) {
      if (b + j < count) sums[b + j] = ex;
      ex += v[j];
    }
    carry += total;
    __syncthreads();
  }
}

__global__ void k_scan_down(uint32_t* __restrict__ a, int64_t count, const uint32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (base + j < count) ? a[base + j] : 0u;
    s += v[j];
  }
  uint32_t total;
  uint32_t ex = block_exclusive_scan(s, &total) + sums[blockIdx.x];
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < count) a[base + j] = ex;
    ex += v[j];
  }
}

static void exclusive_scan(hipStream_t s, uint32_t* a, int64_t count, uint32_t* sums) {
  const int64_t tiles = div_up(count, kScanTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, (const uint32_t*)a, count, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, sums, tiles);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)tiles), dim3(kScanThreads), 0, s, a, count, (const uint32_t*)sums);
}

// ---- dedup and emit -------------------------------------------------------------
__global__ void k_dup_flags(const unsigned long long* __restrict__ keys, int64_t count, uint32_t* __restrict__ f) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride)
    f[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

__global__ void k_dedup_scatter(const unsigned long long* __restrict__ keys, int64_t count,
                                const uint32_t* __restrict__ pos, unsigned long long* __restrict__ out,
                                unsigned long long* m_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) {
    const bool head = (i == 0 || keys[i] != keys[i - 1]);
    if (head) out[pos[i]] = keys[i];
    if (i == count - 1) *m_out = (unsigned long long)pos[i] + (head ? 1ull : 0ull);
  }
}

template <typename O>
__global__ void k_emit_csr(const unsigned long long* __restrict__ keys, const unsigned long long* m_ptr, int64_t n,
                           O* __restrict__ offsets, int32_t* __restrict__ adj, long long* m_user) {
  const int64_t m = (int64_t)*m_ptr;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) {
    const int64_t src = (int64_t)(keys[i] >> 32);
    const int64_t prev = (i == 0) ? -1 : (int64_t)(keys[i - 1] >> 32);
    for (int64_t x = prev + 1; x <= src; ++x) offsets[x] = (O)i;
    adj[i] = (int32_t)(uint32_t)(keys[i] & 0xffffffffull);
  }
  // the rows after the last entry's row (all of them when m = 0), spread
  // over the grid: with vertices in decreasing-degree order they are every
  // isolated vertex
  const int64_t last = m > 0 ? (int64_t)(keys[m - 1] >> 32) : -1;
  for (int64_t x = last + 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x <= n; x += stride) offsets[x] = (O)m;
  if (blockIdx.x == 0 && threadIdx.x == 0 && m_user) *m_user = (long long)m;
}

__global__ void k_copy_u64(const unsigned long long* a, unsigned long long* b) { *b = *a; }

// Bits of a vertex id in [0, n).
static int id_bits(int64_t n) {
  int bits = 1;
  while (bits < 31 && ((int64_t)1 << bits) < n) ++bits;
  return bits;
}

// Stable LSD radix sort of `sorted` 64-bit keys on the low `bits` bits of
// both 32-bit halves (low half first, so the order is by high half, then low
// half); *src holds the result afterwards and *dst the other buffer.
static void radix_sort(hipStream_t s, unsigned long long** src, unsigned long long** dst, int64_t sorted, int bits,
                       uint32_t* hist, uint32_t* sums) {
  std::vector<int> shifts;
  for (int b = 0; b < bits; b += 8) shifts.push_back(b);
  for (int b = 0; b < bits; b += 8) shifts.push_back(32 + b);
  const int64_t tiles = div_up(sorted > 0 ? sorted : 1, kSortTile);
  for (int sh : shifts) {
    const int lowbit = sh >= 32 ? sh - 32 : sh;
    const int width = (bits - lowbit) < 8 ? (bits - lowbit) : 8;
    const uint32_t dmask = (1u << width) - 1u;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)tiles), dim3(kSortThreads), 0, s,
                       (const unsigned long long*)*src, sorted, sh, dmask, hist, tiles);
    exclusive_scan(s, hist, 256 * tiles, sums);
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)tiles), dim3(kSortThreads), 0, s,
                       (const unsigned long long*)*src, *dst, sorted, sh, dmask, (const uint32_t*)hist, tiles);
    unsigned long long* t = *src;
    *src = *dst;
    *dst = t;
  }
}

// ---- degree order ----------------------------------------------------------------
// Sort key of vertex x: (D - min(deg x, D)) in the high half, x in the low
// half, D = 2^bits - 1; ascending keys = decreasing degree, then id.
template <typename O>
__global__ void k_degree_keys(int64_t n, const O* __restrict__ off, int bits, unsigned long long* __restrict__ keys) {
  const int64_t D = ((int64_t)1 << bits) - 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += stride) {
    int64_t d = (int64_t)off[x + 1] - (int64_t)off[x];
    d = d < D ? d : D;
    keys[x] = ((unsigned long long)(D - d) << 32) | (uint32_t)x;
  }
}

// The first x from which every row is empty (offsets ascending): one lane
// searches.
template <typename O>
__global__ void k_active_prefix(int64_t n, const O* __restrict__ off, long long* out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const O m = off[n];
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] == m) hi = mid;
    else lo = mid + 1;
  }
  *out = lo;
}

// orig_of[i] = the vertex in sorted position i; new_of is its inverse.
__global__ void k_order_maps(int64_t n, const unsigned long long* __restrict__ keys, int32_t* __restrict__ orig_of,
                             int32_t* __restrict__ new_of) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const int32_t x = (int32_t)(uint32_t)keys[i];
    orig_of[i] = x;
    new_of[x] = (int32_t)i;
  }
}

// Pairs renumbered by new_of; ids outside [0, n) are kept as they are, so
// the CSR build still reports them.
__global__ void k_renumber_pairs(int64_t n, int64_t k, const int32_t* __restrict__ u, const int32_t* __restrict__ v,
                                 const int32_t* __restrict__ new_of, int32_t* __restrict__ u2,
                                 int32_t* __restrict__ v2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += stride) {
    const int32_t a = u[i], b = v[i];
    u2[i] = (a >= 0 && (int64_t)a < n) ? new_of[a] : a;
    v2[i] = (b >= 0 && (int64_t)b < n) ? new_of[b] : b;
  }
}

struct CsrWs {
  size_t keys = 0, alt = 0, flags = 0, hist = 0, sums = 0, scal = 0, total = 0;
};

static CsrWs csr_ws(int64_t num_pairs) {
  CsrWs W;
  const int64_t E = 2 * num_pairs;
  const int64_t tiles = div_up(E > 0 ? E : 1, kSortTile);
  const int64_t hcount = 256 * tiles;
  size_t off = 0;
  W.keys = off, off += align256((size_t)E * 8 + 8);
  W.alt = off, off += align256((size_t)E * 8 + 8);
  W.flags = off, off += align256((size_t)(E > hcount ? E : hcount) * 4 + 4);
  W.hist = off, off += align256((size_t)hcount * 4);
  W.sums = off, off += align256((size_t)div_up(hcount > E ? hcount : E, kScanTile) * 4 + 4);
  W.scal = off, off += 256;
  W.total = off;
  return W;
}

}  // namespace cc

using namespace cc;

extern "C" {

cc_status cc_csr_workspace_bytes(int64_t n, int64_t num_pairs, size_t* bytes) {
  if (!bytes) return fail(CC_EINVAL, "bytes is NULL");
  if (n < 1 || n > 0x7fffffffLL || num_pairs < 0) return fail(CC_EINVAL, "bad n or num_pairs");
  if (2 * num_pairs >= 0xffffffffLL) return fail(CC_EINVAL, "more than 2^32-1 directed edges");
  *bytes = csr_ws(num_pairs).total;
  return CC_OK;
}

cc_status cc_build_csr(cc_ctx* ctx, int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v, int dedup,
                       void* workspace, size_t ws_bytes, void* offsets_out, int offsets_64bit, int32_t* adj_out,
                       int64_t* m_dev, void* hip_stream) {
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  if (n < 1 || n > 0x7fffffffLL || num_pairs < 0) return fail(CC_EINVAL, "bad n or num_pairs");
  if (2 * num_pairs >= 0xffffffffLL) return fail(CC_EINVAL, "more than 2^32-1 directed edges");
  if (!offsets_64bit && 2 * num_pairs > 0x7fffffffLL) return fail(CC_EINVAL, "edge count needs 64-bit offsets");
  if (!offsets_out || (num_pairs > 0 && (!u || !v || !adj_out))) return fail(CC_EINVAL, "NULL array argument");
  const CsrWs W = csr_ws(num_pairs);
  if (!workspace || ws_bytes < W.total)
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, W.total);
  if (((uintptr_t)workspace & 255u) != 0) return fail(CC_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)hip_stream;
  char* w = (char*)workspace;
  unsigned long long* keys = (unsigned long long*)(w + W.keys);
  unsigned long long* alt = (unsigned long long*)(w + W.alt);
  uint32_t* flags = (uint32_t*)(w + W.flags);
  uint32_t* hist = (uint32_t*)(w + W.hist);
  uint32_t* sums = (uint32_t*)(w + W.sums);
  unsigned long long* scal = (unsigned long long*)(w + W.scal);  // [0] = E, [1] = m

  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t*)scal, (int64_t)8, 0u);
  if (num_pairs > 0)
    hipLaunchKernelGGL(k_expand_pairs, dim3(grid_for(num_pairs, 256, 8192)), dim3(256), 0, s, n, num_pairs, u, v,
                       keys, scal, ctx->dev);
  CC_LAUNCH_CHECK();
  unsigned long long E = 0;
  CC_HIP(hipMemcpyAsync(&E, scal, 8, hipMemcpyDeviceToHost, s));
  CC_HIP(hipStreamSynchronize(s));

  const int bits = id_bits(n);
  const int64_t count = (int64_t)E;          // real keys; they sort ahead of the sentinels
  const int64_t sorted = 2 * num_pairs;       // keys the radix passes move
  unsigned long long* src = keys;
  unsigned long long* dst = alt;
  if (count > 0) radix_sort(s, &src, &dst, sorted, bits, hist, sums);
  CC_LAUNCH_CHECK();
  const unsigned long long* final_keys = src;
  if (count > 0 && dedup) {
    hipLaunchKernelGGL(k_dup_flags, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s,
                       (const unsigned long long*)src, count, flags);
    exclusive_scan(s, flags, count, sums);
    hipLaunchKernelGGL(k_dedup_scatter, dim3(grid_for(count, 256, 8192)), dim3(256), 0, s,
                       (const unsigned long long*)src, count, (const uint32_t*)flags, dst, scal + 1);
    final_keys = dst;
  } else {
    hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(1), 0, s, (const unsigned long long*)scal, scal + 1);
  }
  if (offsets_64bit)
    hipLaunchKernelGGL(k_emit_csr<int64_t>, dim3(grid_for(count + 1, 256, 8192)), dim3(256), 0, s, final_keys,
                       (const unsigned long long*)(scal + 1), n, (int64_t*)offsets_out, adj_out, (long long*)m_dev);
  else
    hipLaunchKernelGGL(k_emit_csr<int32_t>, dim3(grid_for(count + 1, 256, 8192)), dim3(256), 0, s, final_keys,
                       (const unsigned long long*)(scal + 1), n, (int32_t*)offsets_out, adj_out, (long long*)m_dev);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

// Workspace of cc_build_csr_degree_order: one CSR build's workspace sized
// for max(num_pairs, ceil(n / 2)) pairs (its sort buffers also sort the n
// vertex keys), then the renumbered pair list.
static size_t degree_order_ws(int64_t n, int64_t num_pairs, size_t* csr_part) {
  const int64_t big = num_pairs > (n + 1) / 2 ? num_pairs : (n + 1) / 2;
  *csr_part = csr_ws(big).total;
  return *csr_part + 2 * align256((size_t)(num_pairs > 0 ? num_pairs : 1) * 4);
}

cc_status cc_csr_degree_order_workspace_bytes(int64_t n, int64_t num_pairs, size_t* bytes) {
  if (!bytes) return fail(CC_EINVAL, "bytes is NULL");
  if (n < 1 || n > 0x7fffffffLL || num_pairs < 0) return fail(CC_EINVAL, "bad n or num_pairs");
  if (2 * num_pairs >= 0xffffffffLL) return fail(CC_EINVAL, "more than 2^32-1 directed edges");
  size_t part = 0;
  *bytes = degree_order_ws(n, num_pairs, &part);
  return CC_OK;
}

cc_status cc_build_csr_degree_order(cc_ctx* ctx, int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v,
                                    int dedup, void* workspace, size_t ws_bytes, void* offsets_out, int offsets_64bit,
                                    int32_t* adj_out, int64_t* m_dev, int32_t* orig_of, int32_t* new_of,
                                    void* hip_stream) {
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  if (n < 1 || n > 0x7fffffffLL || num_pairs < 0) return fail(CC_EINVAL, "bad n or num_pairs");
  if (!orig_of || !new_of) return fail(CC_EINVAL, "NULL permutation argument");
  size_t part = 0;
  const size_t need = degree_order_ws(n, num_pairs, &part);
  if (!workspace || ws_bytes < need)
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
  if (((uintptr_t)workspace & 255u) != 0) return fail(CC_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = (hipStream_t)hip_stream;
  // 1. the CSR in the given numbering, for the degrees
  cc_status st = cc_build_csr(ctx, n, num_pairs, u, v, dedup, workspace, part, offsets_out, offsets_64bit, adj_out,
                              m_dev, hip_stream);
  if (st != CC_OK) return st;
  // 2. vertices sorted by decreasing degree, then id (the build's sort buffers)
  const int64_t big = num_pairs > (n + 1) / 2 ? num_pairs : (n + 1) / 2;
  const CsrWs W = csr_ws(big);
  char* w = (char*)workspace;
  unsigned long long* src = (unsigned long long*)(w + W.keys);
  unsigned long long* dst = (unsigned long long*)(w + W.alt);
  const int bits = id_bits(n);
  if (offsets_64bit)
    hipLaunchKernelGGL(k_degree_keys<int64_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n,
                       (const int64_t*)offsets_out, bits, src);
  else
    hipLaunchKernelGGL(k_degree_keys<int32_t>, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n,
                       (const int32_t*)offsets_out, bits, src);
  radix_sort(s, &src, &dst, n, bits, (uint32_t*)(w + W.hist), (uint32_t*)(w + W.sums));
  hipLaunchKernelGGL(k_order_maps, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n,
                     (const unsigned long long*)src, orig_of, new_of);
  CC_LAUNCH_CHECK();
  if (num_pairs == 0) return CC_OK;  // no edges: every vertex has degree 0, the CSR is the same
  // 3. the pairs renumbered, and the CSR built again from them
  int32_t* u2 = (int32_t*)(w + part);
  int32_t* v2 = (int32_t*)(w + part + align256((size_t)num_pairs * 4));
  hipLaunchKernelGGL(k_renumber_pairs, dim3(grid_for(num_pairs, 256, 8192)), dim3(256), 0, s, n, num_pairs, u, v,
                     (const int32_t*)new_of, u2, v2);
  CC_LAUNCH_CHECK();
  return cc_build_csr(ctx, n, num_pairs, u2, v2, dedup, workspace, part, offsets_out, offsets_64bit, adj_out, m_dev,
                      hip_stream);
}

cc_status cc_csr_active_prefix(int64_t n, const void* offsets, int offsets_are_64bit, int64_t* active_dev,
                               void* hip_stream) {
  if (n < 1 || n > 0x7fffffffLL) return fail(CC_EINVAL, "bad n");
  if (!offsets || !active_dev) return fail(CC_EINVAL, "NULL pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  if (offsets_are_64bit)
    hipLaunchKernelGGL(k_active_prefix<int64_t>, dim3(1), dim3(64), 0, s, n, (const int64_t*)offsets,
                       (long long*)active_dev);
  else
    hipLaunchKernelGGL(k_active_prefix<int32_t>, dim3(1), dim3(64), 0, s, n, (const int32_t*)offsets,
                       (long long*)active_dev);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

}  // extern "C"
