// Approximate minimum spanning forest (ConnectIt Section 5.1, "Approximate
// Minimum Spanning Forest").
//
// Edges are bucketed by weight with boundaries t_0 = W_min and
// t_{i+1} = t_i (1 + eps) (double product rounded down to float, so every
// bucket spans a ratio of at most 1 + eps) and the buckets are taken in
// increasing order, each adding a spanning forest of its edges over the
// components of the earlier ones.  That is Kruskal's algorithm on weights
// rounded down to their bucket boundary, hence a (1 + eps)-approximate
// minimum spanning forest.
//
// The buckets fall into two phases.
//  * Light buckets, the first ones, holding about a requested share of the
//    entries (chosen from a sample of the weights): one pass over the CSR
//    counts, per block and bucket, the entries (u, v) with u < v, and a
//    second identical pass scatters them into a bucket-sorted edge list at
//    offsets from a scan of those counts (no contended atomics, the same
//    layout every run).  Each light bucket is then one union launch over its
//    slice, and runs of small buckets share one single-block launch with a
//    block barrier between buckets.  Early buckets hold few edges; this way
//    each light edge is read once rather than in every round.
//  * Every later bucket is a round of the paper's sampled no-filter variant
//    (AMSF-NF-S): the rows of the vertices outside the largest component of
//    the labelling are scanned, and entries of the round's bucket are united.
//    A vertex of the largest component is skipped; its edges to other
//    components are seen from their other endpoint.  The largest component
//    and the candidate lists are refreshed once enough edges have been added
//    since the last refresh (skipping a stale one stays correct, since
//    components only grow).
//
// Union-find is UF-Rem-CAS with SplitAtomicOne and FindNaive, the paper's
// choice for this application; the edge that hooks a root is recorded at
// that root's slot, with its weight.
#include <algorithm>
#include <cmath>

#include "cc_frontier.h"
#include "cc_static.h"

namespace cc {

constexpr int kAmsfMaxBuckets = 4096;   // bucket table size (LDS)
constexpr int kAmsfLightMax = 1024;     // light buckets at most
constexpr int kAmsfTile = 4096;         // adjacency entries per tile of the two passes
constexpr int kAmsfThreads = 512;       // block of the two passes
constexpr int kAmsfPassGrid = 768;      // blocks of the two passes (3 per CU; at most 2048)
constexpr int kAmsfRangeGrid = 1024;    // blocks of the weight-range pass
constexpr int kAmsfSamples = 16384;     // weights sampled to pick the light buckets
constexpr int kAmsfSeqMax = 2048;       // buckets this small share a single-block launch
constexpr int kAmsfSeqThreads = 1024;
constexpr uint64_t kTagAmsf = 0x616d7366ULL;  // "amsf"

struct AmsfScalars {
  float wmin, wmax;
  uint32_t bad;          // entries whose weight is not finite and > 0
  uint32_t too_many;     // the weight range needs more than kAmsfMaxBuckets buckets
  int32_t nb;            // buckets (0: no entries, or an error above)
  int32_t b0;            // light buckets picked from the sample
  float log2_wmin;
  float inv_log2_ratio;  // 1 / log2(1 + eps)
  uint32_t pad[56];      // to 256 bytes
};
static_assert(sizeof(AmsfScalars) == 256, "AmsfScalars is one 256-byte block");

// Device block copied to the host in one transfer after the first pass.
struct AmsfHostBlock {
  AmsfScalars sc;
  long long lstart[kAmsfLightMax + 1];  // start of each light bucket in the sorted list, then the total
  long long rowsum[kAmsfLightMax];      // light entries (u < v) per bucket
  uint32_t shist[kAmsfMaxBuckets];      // sampled entries per bucket (kAmsfSamples in all)
};

// ---- weight range --------------------------------------------------------

struct RangePart {
  float lo, hi;
  uint32_t bad;
  uint32_t pad;
};

__device__ __forceinline__ void range_add(float x, float& lo, float& hi, uint32_t& bad) {
  // x > 0 and finite; NaN fails the first test
  if (!(x > 0.0f) || !(x <= 3.402823466e38f)) {
    ++bad;
    return;
  }
  lo = fminf(lo, x);
  hi = fmaxf(hi, x);
}

__global__ void __launch_bounds__(kFBlock) k_amsf_range(int64_t m, const float* __restrict__ w, int aligned,
                                                        RangePart* __restrict__ part) {
  __shared__ float slo[kFBlock / kWave], shi[kFBlock / kWave];
  __shared__ uint32_t sbad[kFBlock / kWave];
  float lo = INFINITY, hi = 0.0f;
  uint32_t bad = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (aligned) {
    const int64_t q = m / 4;
    // four 16-byte loads in flight per thread
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < q; i += 4 * stride) {
      float4 x[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        x[k] = i + k * stride < q ? ((const float4*)w)[i + k * stride] : make_float4(1.0f, 1.0f, 1.0f, 1.0f);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (i + k * stride >= q) continue;
        range_add(x[k].x, lo, hi, bad);
        range_add(x[k].y, lo, hi, bad);
        range_add(x[k].z, lo, hi, bad);
        range_add(x[k].w, lo, hi, bad);
      }
    }
    for (int64_t i = 4 * q + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride)
      range_add(w[i], lo, hi, bad);
  } else {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += stride) range_add(w[i], lo, hi, bad);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, kWave));
    hi = fmaxf(hi, __shfl_xor(hi, o, kWave));
    bad += __shfl_xor(bad, o, kWave);
  }
  const int wv = threadIdx.x / kWave;
  if (lane_id() == 0) {
    slo[wv] = lo;
    shi[wv] = hi;
    sbad[wv] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kFBlock / kWave; ++i) {
      lo = fminf(lo, slo[i]);
      hi = fmaxf(hi, shi[i]);
      bad += sbad[i];
    }
    part[blockIdx.x] = RangePart{lo, hi, bad, 0u};
  }
}

// Largest bucket b < nb with t[b] <= x (x >= t[0]): a logarithm gives a
// first guess, exact comparisons with the table settle it.
__device__ __forceinline__ int bucket_of(float x, const float* t, int nb, float log2_wmin, float inv_log2_ratio) {
  int b = (int)((__log2f(x) - log2_wmin) * inv_log2_ratio);
  b = b < 0 ? 0 : (b >= nb ? nb - 1 : b);
  while (b > 0 && t[b] > x) --b;
  while (b + 1 < nb && t[b + 1] <= x) ++b;
  return b;
}

// One block: the range, the bucket boundaries, and the light buckets from a
// sample of the weights.  b0 is the largest b whose earlier buckets hold at
// most light_fraction of the sampled entries (0 when light_fraction is 0).
__global__ void __launch_bounds__(1024) k_amsf_setup(const RangePart* __restrict__ part, int nparts, double eps,
                                                     float light_fraction, uint64_t key, int64_t m,
                                                     const float* __restrict__ w, float* __restrict__ thr,
                                                     AmsfScalars* as, uint32_t* __restrict__ shist) {
  __shared__ float slo[1024 / kWave], shi[1024 / kWave];
  __shared__ uint32_t sbad[1024 / kWave];
  __shared__ uint32_t hist[kAmsfMaxBuckets];
  __shared__ float ts[kAmsfMaxBuckets + 1];
  __shared__ int32_t s_nb;
  float lo = INFINITY, hi = 0.0f;
  uint32_t bad = 0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
    lo = fminf(lo, part[i].lo);
    hi = fmaxf(hi, part[i].hi);
    bad += part[i].bad;
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fminf(lo, __shfl_xor(lo, o, kWave));
    hi = fmaxf(hi, __shfl_xor(hi, o, kWave));
    bad += __shfl_xor(bad, o, kWave);
  }
  const int wv = threadIdx.x / kWave;
  if (lane_id() == 0) {
    slo[wv] = lo;
    shi[wv] = hi;
    sbad[wv] = bad;
  }
  for (int i = threadIdx.x; i < kAmsfMaxBuckets; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 1024 / kWave; ++i) {
      lo = fminf(lo, slo[i]);
      hi = fmaxf(hi, shi[i]);
      bad += sbad[i];
    }
    int32_t nb = 0;
    uint32_t too_many = 0;
    if (bad == 0 && m > 0) {
      thr[0] = lo;
      float t = lo;
      while (t <= hi) {
        if (nb == kAmsfMaxBuckets) {
          too_many = 1;
          break;
        }
        t = __double2float_rd((double)t * (1.0 + eps));
        thr[++nb] = t;
      }
      if (too_many) nb = 0;
    }
    as->wmin = lo;
    as->wmax = hi;
    as->bad = bad;
    as->too_many = too_many;
    as->nb = nb;
    as->log2_wmin = __log2f(lo);
    as->inv_log2_ratio = (float)(1.0 / log2(1.0 + eps));
    s_nb = nb;
  }
  __syncthreads();
  const int nb = s_nb;
  if (nb == 0) {
    if (threadIdx.x == 0) as->b0 = 0;
    return;
  }
  const float l2 = as->log2_wmin, ilr = as->inv_log2_ratio;
  for (int i = threadIdx.x; i <= nb; i += blockDim.x) ts[i] = thr[i];
  __syncthreads();
  for (int i = threadIdx.x; i < kAmsfSamples; i += blockDim.x) {
    const int64_t j = (int64_t)(sm_out(key, (uint64_t)i) % (uint64_t)m);
    atomicAdd(&hist[bucket_of(w[j], ts, nb, l2, ilr)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x) shist[i] = hist[i];
  if (threadIdx.x == 0 && light_fraction <= 0.0f) as->b0 = 0;
  if (threadIdx.x == 0 && light_fraction > 0.0f) {
    const double budget = (double)light_fraction * kAmsfSamples;
    int32_t b0 = 0;
    uint32_t below = 0;  // samples in buckets < b0
    while (b0 < nb && b0 < kAmsfLightMax && (double)(below + hist[b0]) <= budget) below += hist[b0++];
    as->b0 = b0;
  }
}

// ---- the two passes over the CSR -------------------------------------------

// tile_row[k] = the row holding adjacency entry k * kAmsfTile.
template <typename I>
__global__ void __launch_bounds__(kFBlock) k_amsf_tile_rows(int64_t n, const I* __restrict__ off,
                                                            int32_t* __restrict__ tile_row) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; u < n; u += stride) {
    const int64_t s = off[u], e = off[u + 1];
    for (int64_t k = (s + kAmsfTile - 1) / kAmsfTile; k * kAmsfTile < e; ++k) tile_row[k] = (int32_t)u;
  }
}

// The light entries of the CSR, in two identical passes.  A block takes one
// tile of kAmsfTile entries at a time; each thread owns kAmsfPer consecutive
// entries.  Row ids come from the tile's row starts: every row r that begins
// inside the tile marks its first position with r (atomicMax, so that of
// several rows starting at one position the last, the non-empty one, wins),
// and a block-wide running maximum carries the row to every entry; empty
// rows cost nothing more.  The next tile's entries are loaded while the
// current one is processed.
//
// Pass A (SCATTER false): per block, the light entries (weight below t[b0])
// (u, v) with u < v of each light bucket into lpart[b * gridDim.x + block].
// Pass B (SCATTER true): the same entries in the same blocks; each goes to
// the sorted list at lstart[b] + lpart[b][block] (lpart scanned along each
// bucket) plus its place inside the block.  b0_arg < 0: read b0 from the
// device scalars.
constexpr int kAmsfPer = kAmsfTile / kAmsfThreads;  // 8 entries per thread and tile
static_assert(kAmsfPer == 8, "two 16-byte loads per thread");

// A thread's kAmsfPer weights and neighbours of one tile (+inf weight past
// the end of the adjacency).
struct PassChunk {
  float x[kAmsfPer];
  int32_t v[kAmsfPer];
};

__device__ __forceinline__ void load_chunk(PassChunk& c, int64_t c0, int64_t E1, const float* w, const int32_t* adj,
                                           int aligned) {
  if (aligned && c0 + kAmsfPer <= E1) {
    const float4 a0 = *(const float4*)(w + c0), a1 = *(const float4*)(w + c0 + 4);
    const int4 b0 = *(const int4*)(adj + c0), b1 = *(const int4*)(adj + c0 + 4);
    c.x[0] = a0.x, c.x[1] = a0.y, c.x[2] = a0.z, c.x[3] = a0.w;
    c.x[4] = a1.x, c.x[5] = a1.y, c.x[6] = a1.z, c.x[7] = a1.w;
    c.v[0] = b0.x, c.v[1] = b0.y, c.v[2] = b0.z, c.v[3] = b0.w;
    c.v[4] = b1.x, c.v[5] = b1.y, c.v[6] = b1.z, c.v[7] = b1.w;
  } else {
#pragma unroll
    for (int i = 0; i < kAmsfPer; ++i) {
      const bool in = c0 + i < E1;
      c.x[i] = in ? w[c0 + i] : INFINITY;
      c.v[i] = in ? adj[c0 + i] : 0;
    }
  }
}

template <typename I, bool SCATTER>
__global__ void __launch_bounds__(kAmsfThreads) k_amsf_pass(int64_t n, int64_t m, const I* __restrict__ off,
                                                            const int32_t* __restrict__ adj,
                                                            const float* __restrict__ w,
                                                            const float* __restrict__ thr, const AmsfScalars* as,
                                                            const int32_t* __restrict__ tile_row, int64_t ntiles,
                                                            int32_t b0_arg, long long* __restrict__ lpart,
                                                            const long long* __restrict__ lstart,
                                                            int2* __restrict__ luv, float* __restrict__ lw,
                                                            int aligned) {
  __shared__ float t[kAmsfLightMax + 1];
  __shared__ int32_t starts[kAmsfTile];
  __shared__ int32_t lcnt[kAmsfLightMax];
  __shared__ int32_t wmax[kAmsfThreads / kWave];
  const int nb = as->nb;
  const int b0 = nb == 0 ? 0 : (b0_arg >= 0 ? b0_arg : as->b0);
  if (b0 == 0) return;
  const float l2 = as->log2_wmin, ilr = as->inv_log2_ratio;
  for (int i = threadIdx.x; i <= b0; i += blockDim.x) t[i] = thr[i];
  for (int i = threadIdx.x; i < b0; i += blockDim.x) lcnt[i] = 0;
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  int64_t k = blockIdx.x;
  PassChunk cur, nxt;
  int32_t r0 = 0, r1 = 0, nr0 = 0, nr1 = 0;
  if (k < ntiles) {
    const int64_t E0 = k * kAmsfTile, E1 = (E0 + kAmsfTile < m) ? E0 + kAmsfTile : m;
    r0 = tile_row[k];
    r1 = (k + 1 < ntiles) ? tile_row[k + 1] : (int32_t)(n - 1);
    load_chunk(cur, E0 + (int64_t)kAmsfPer * threadIdx.x, E1, w, adj, aligned);
  }
  __syncthreads();
  const float tb0 = t[b0];
  for (; k < ntiles; k += gridDim.x) {
    const int64_t E0 = k * kAmsfTile;
    const int64_t E1 = (E0 + kAmsfTile < m) ? E0 + kAmsfTile : m;
    for (int i = threadIdx.x; i < kAmsfTile; i += blockDim.x) starts[i] = -1;
    const int64_t kn = k + gridDim.x;
    if (kn < ntiles) {
      const int64_t F0 = kn * kAmsfTile, F1 = (F0 + kAmsfTile < m) ? F0 + kAmsfTile : m;
      nr0 = tile_row[kn];
      nr1 = (kn + 1 < ntiles) ? tile_row[kn + 1] : (int32_t)(n - 1);
      load_chunk(nxt, F0 + (int64_t)kAmsfPer * threadIdx.x, F1, w, adj, aligned);
    }
    __syncthreads();
    if (threadIdx.x == 0) atomicMax(&starts[0], r0);
    for (int64_t r = (int64_t)r0 + 1 + threadIdx.x; r <= r1; r += blockDim.x) {
      const int64_t o = (int64_t)off[r];
      if (o < E1) atomicMax(&starts[o - E0], (int32_t)r);
    }
    __syncthreads();
    // running maximum over the tile: thread-local over its kAmsfPer
    // positions, then an exclusive maximum over the threads before it
    int32_t row[kAmsfPer];
    int32_t run = -1;
#pragma unroll
    for (int i = 0; i < kAmsfPer; ++i) {
      const int32_t sv = starts[kAmsfPer * threadIdx.x + i];
      run = sv > run ? sv : run;
      row[i] = run;
    }
    int32_t inc = run;
    for (int o = 1; o < kWave; o <<= 1) {
      const int32_t y = __shfl_up(inc, o, kWave);
      if (lane >= o) inc = y > inc ? y : inc;
    }
    if (lane == kWave - 1) wmax[wv] = inc;
    int32_t carry = __shfl_up(inc, 1, kWave);
    if (lane == 0) carry = -1;
    __syncthreads();
    for (int q = 0; q < wv; ++q) carry = wmax[q] > carry ? wmax[q] : carry;
    const int64_t c0 = E0 + (int64_t)kAmsfPer * threadIdx.x;
#pragma unroll
    for (int i = 0; i < kAmsfPer; ++i) {
      const int32_t u = row[i] > carry ? row[i] : carry;
      if (c0 + i < E1 && cur.x[i] < tb0 && u < cur.v[i]) {
        const int b = bucket_of(cur.x[i], t, b0, l2, ilr);
        const int32_t q = atomicAdd(&lcnt[b], 1);
        if (SCATTER) {
          const long long p = lstart[b] + lpart[(int64_t)b * gridDim.x + blockIdx.x] + q;
          luv[p] = make_int2(u, cur.v[i]);
          lw[p] = cur.x[i];
        }
      }
    }
    __syncthreads();
    cur = nxt;
    r0 = nr0;
    r1 = nr1;
  }
  if (!SCATTER)
    for (int i = threadIdx.x; i < b0; i += blockDim.x) lpart[(int64_t)i * gridDim.x + blockIdx.x] = lcnt[i];
}

// Block b < b0: exclusive scan of bucket b's per-block counts (G <= 2048,
// two consecutive counts per thread) in place, the bucket's total to
// rowsum[b].
__global__ void __launch_bounds__(1024) k_amsf_row_scan(long long* lpart, int G, const AmsfScalars* as,
                                                        long long* __restrict__ rowsum) {
  __shared__ long long wsum[1024 / kWave];
  const int b = blockIdx.x;
  if (as->nb == 0 || b >= as->b0) return;
  const int t = threadIdx.x, lane = lane_id(), wv = t / kWave;
  long long* row = lpart + (int64_t)b * G;
  const long long x0 = 2 * t < G ? row[2 * t] : 0;
  const long long x1 = 2 * t + 1 < G ? row[2 * t + 1] : 0;
  const long long x = x0 + x1;
  long long inc = x;
  for (int o = 1; o < kWave; o <<= 1) {
    const long long y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) wsum[wv] = inc;
  __syncthreads();
  long long before = 0, total = 0;
  for (int q = 0; q < 1024 / kWave; ++q) {
    if (q < wv) before += wsum[q];
    total += wsum[q];
  }
  const long long ex = before + inc - x;
  if (2 * t < G) row[2 * t] = ex;
  if (2 * t + 1 < G) row[2 * t + 1] = ex + x0;
  if (t == 0) rowsum[b] = total;
}

// One block: lstart[b] = sum of rowsum[b'] for b' < b, lstart[b0] = total.
__global__ void __launch_bounds__(1024) k_amsf_lstart(const AmsfScalars* as, const long long* __restrict__ rowsum,
                                                      long long* __restrict__ lstart) {
  __shared__ long long wsum[1024 / kWave];
  const int b0 = as->nb > 0 ? as->b0 : 0;
  const int t = threadIdx.x, lane = lane_id(), wv = t / kWave;
  const long long x = t < b0 ? rowsum[t] : 0;
  long long inc = x;
  for (int o = 1; o < kWave; o <<= 1) {
    const long long y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) wsum[wv] = inc;
  __syncthreads();
  long long before = 0, total = 0;
  for (int q = 0; q < 1024 / kWave; ++q) {
    if (q < wv) before += wsum[q];
    total += wsum[q];
  }
  if (t < b0) lstart[t] = before + inc - x;
  if (t == 0) lstart[b0] = total;
}

// ---- unions ------------------------------------------------------------------

__global__ void k_amsf_iota(int64_t n, int32_t* __restrict__ P) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) P[i] = (int32_t)i;
}

__device__ __forceinline__ void amsf_unite(int32_t* P, int32_t u, int32_t v, float x, int2* hook, float* hookw) {
  const int32_t r = union_rem<kSplitOne, kFindNaive>(P, u, v);
  if (r >= 0) {
    hook[r] = make_int2(u, v);
    hookw[r] = x;
  }
}

// Light buckets [b_lo, b_hi) in order, one block, a barrier between buckets
// (every union of a bucket has returned before the next bucket starts).
__global__ void __launch_bounds__(kAmsfSeqThreads) k_amsf_light_seq(const int2* __restrict__ luv,
                                                                    const float* __restrict__ lw,
                                                                    const long long* __restrict__ lstart, int b_lo,
                                                                    int b_hi, int32_t* P, int2* hook, float* hookw) {
  for (int b = b_lo; b < b_hi; ++b) {
    const long long s = lstart[b], e = lstart[b + 1];
    for (long long i = s + threadIdx.x; i < e; i += blockDim.x) {
      const int2 uv = luv[i];
      amsf_unite(P, uv.x, uv.y, lw[i], hook, hookw);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kFBlock) k_amsf_light(const int2* __restrict__ luv, const float* __restrict__ lw,
                                                        long long s, long long e, int32_t* P, int2* hook,
                                                        float* hookw) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (long long i = s + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < e; i += stride) {
    const int2 uv = luv[i];
    amsf_unite(P, uv.x, uv.y, lw[i], hook, hookw);
  }
}

// One no-filter round over the candidate rows: entries of bucket b.
struct AmsfRoundOp {
  int32_t* P;
  const float* w;
  const float* thr;
  int32_t b;
  int2* hook;
  float* hookw;
  __device__ __forceinline__ bool operator()(int32_t u, int32_t v, int64_t j) const {
    const float x = w[j];
    if (x < thr[b] || !(x < thr[b + 1])) return false;
    amsf_unite(P, u, v, x, hook, hookw);
    return false;
  }
};

// One round over the low-degree candidates (degree <= kThrWave, one thread
// each), fused with the largest-component test: a candidate whose root is
// now the root of L_max is dropped (its edges to other components are seen
// from their other endpoints); the others visit their entries of bucket b
// and stay on the list for the next round.  Each block takes kAmsfRoundTile
// consecutive list entries and appends its survivors with one atomic.  The
// list lengths rotate through three counters: round r reads cnt[r % 3],
// appends to cnt[(r + 1) % 3] and clears cnt[(r + 2) % 3] for round r + 1.
constexpr int kAmsfRoundThreads = 1024;
constexpr int kAmsfRoundPer = 4;
constexpr int kAmsfRoundTile = kAmsfRoundThreads * kAmsfRoundPer;

template <typename I>
__global__ void __launch_bounds__(kAmsfRoundThreads) k_amsf_round(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                                  uint32_t* cnt, int r, const I* __restrict__ off,
                                                                  const int32_t* __restrict__ adj,
                                                                  const float* __restrict__ w,
                                                                  const float* __restrict__ thr, int b, int32_t* P,
                                                                  int32_t L, int2* hook, float* hookw) {
  __shared__ int32_t wsum[kAmsfRoundThreads / kWave];
  __shared__ uint32_t s_base;
  const uint32_t c = cnt[r % 3];
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[(r + 2) % 3] = 0u;
  const int64_t base = (int64_t)blockIdx.x * kAmsfRoundTile;
  if (base >= (int64_t)c) return;
  const float lo = thr[b], hi = thr[b + 1];
  __shared__ int32_t s_lroot;
  if (threadIdx.x == 0) s_lroot = find_naive(P, L);
  // the loads of a thread's kAmsfRoundPer candidates are issued stage by
  // stage, so that their latencies overlap
  int32_t u[kAmsfRoundPer], p[kAmsfRoundPer], pp[kAmsfRoundPer];
#pragma unroll
  for (int q = 0; q < kAmsfRoundPer; ++q) {
    const int64_t i = base + q * kAmsfRoundThreads + threadIdx.x;
    u[q] = i < (int64_t)c ? in[i] : -1;
  }
#pragma unroll
  for (int q = 0; q < kAmsfRoundPer; ++q) p[q] = u[q] >= 0 ? ld(P + u[q]) : -1;
#pragma unroll
  for (int q = 0; q < kAmsfRoundPer; ++q) pp[q] = (u[q] >= 0 && p[q] != u[q]) ? ld(P + p[q]) : p[q];
  __syncthreads();
  const int32_t lroot = s_lroot;
  int32_t keep[kAmsfRoundPer];
  int64_t rs[kAmsfRoundPer], re[kAmsfRoundPer];
  int nk = 0;
#pragma unroll
  for (int q = 0; q < kAmsfRoundPer; ++q) {
    keep[q] = -1;
    rs[q] = re[q] = 0;
    if (u[q] < 0) continue;
    int32_t ru = p[q];
    if (p[q] != u[q]) {
      ru = pp[q] == p[q] ? p[q] : find_naive(P, pp[q]);
      if (ru != p[q]) st(P + u[q], ru);  // shortcut, as the compress step would
    }
    if (ru == lroot) continue;
    keep[q] = u[q];
    ++nk;
  }
#pragma unroll
  for (int q = 0; q < kAmsfRoundPer; ++q)
    if (keep[q] >= 0) {
      rs[q] = (int64_t)off[keep[q]];
      re[q] = (int64_t)off[keep[q] + 1];
    }
#pragma unroll
  for (int q = 0; q < kAmsfRoundPer; ++q)
    for (int64_t j = rs[q]; j < re[q]; ++j) {
      const float x = w[j];
      if (x >= lo && x < hi) amsf_unite(P, keep[q], adj[j], x, hook, hookw);
    }
  // block-wide exclusive scan of the survivors, one atomic per block
  const int lane = lane_id(), wv = threadIdx.x / kWave;
  int32_t inc = nk;
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) wsum[wv] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t tot = 0;
    for (int q = 0; q < kAmsfRoundThreads / kWave; ++q) {
      const int32_t x = wsum[q];
      wsum[q] = (int32_t)tot;
      tot += (uint32_t)x;
    }
    s_base = tot ? atomicAdd(cnt + (r + 1) % 3, tot) : 0u;
  }
  __syncthreads();
  uint32_t pos = s_base + (uint32_t)wsum[wv] + (uint32_t)(inc - nk);
#pragma unroll
  for (int q = 0; q < kAmsfRoundPer; ++q)
    if (keep[q] >= 0) out[pos++] = keep[q];
}

// Round counters: the thread-bin candidate count into cnt[0], the others 0.
__global__ void k_amsf_round_init(const DevScalars* sc, uint32_t* cnt) {
  cnt[0] = (uint32_t)sc->bin_count[0];
  cnt[1] = 0u;
  cnt[2] = 0u;
}

// ---- total weight --------------------------------------------------------------

__global__ void __launch_bounds__(kFBlock) k_amsf_weight(const float* __restrict__ ew, const long long* num_edges,
                                                         double* __restrict__ part) {
  __shared__ double red[kFBlock / kWave];
  const long long k = *num_edges;
  double s = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < k; i += stride) s += (double)ew[i];
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kFBlock / kWave; ++i) s += red[i];
    part[blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(kFBlock) k_amsf_weight_sum(const double* __restrict__ part, int nparts,
                                                             double* out) {
  __shared__ double red[kFBlock / kWave];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
  s = wave_sum(s);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kFBlock / kWave; ++i) s += red[i];
    *out = s;
  }
}

constexpr int kAmsfWeightGrid = 1024;

// ---- host ------------------------------------------------------------------------

static cc_variant amsf_variant() {
  cc_variant v{};
  cc_default_variant(&v);
  v.sample = CC_SAMPLE_NONE;
  v.finish = CC_FIN_UF_REM_CAS;
  v.splice = CC_SPLICE_SPLIT_ONE;
  v.find = CC_FIND_NAIVE;
  return v;
}

static int64_t amsf_light_cap(int64_t m, float f) {
  if (!(f > 0.0f)) return 0;
  const double c = 2.0 * (double)f * (double)m + 65536.0;
  return c < (double)m ? (int64_t)c : m;
}

struct AmsfLayout {
  size_t hook = 0, hookw = 0, fcnt = 0, hostblk = 0, thr = 0, range = 0, tile_row = 0, lpart = 0, luv = 0,
         lw = 0, wpart = 0, total = 0;
  int64_t cap = 0, ntiles = 0;
};

static AmsfLayout amsf_layout(int64_t n, int64_t m, float f) {
  AmsfLayout L;
  const cc_variant v = amsf_variant();
  size_t off = align256(ws_layout(n, m, &v).total);
  L.ntiles = (m + kAmsfTile - 1) / kAmsfTile;
  L.cap = amsf_light_cap(m, f);
  L.hook = off, off += align256((size_t)n * 8);
  L.hookw = off, off += align256((size_t)n * 4);
  L.fcnt = off, off += align256((size_t)forest_tiles(n) * 4);
  L.hostblk = off, off += align256(sizeof(AmsfHostBlock));
  L.thr = off, off += align256((kAmsfMaxBuckets + 1) * 4);
  L.range = off, off += align256(kAmsfRangeGrid * sizeof(RangePart));
  L.tile_row = off, off += align256((size_t)(L.ntiles + 1) * 4);
  L.lpart = off, off += align256((size_t)kAmsfLightMax * kAmsfPassGrid * 8);
  L.luv = off, off += align256((size_t)L.cap * 8);
  L.lw = off, off += align256((size_t)L.cap * 4);
  L.wpart = off, off += align256(kAmsfWeightGrid * 8);
  L.total = off;
  return L;
}

static cc_status check_amsf_options(const cc_amsf_options* opt) {
  if (!opt) return fail(CC_EINVAL, "options are NULL");
  if (!(opt->epsilon >= 0x1p-20f && opt->epsilon <= 0x1p20f))
    return fail(CC_EINVAL, "epsilon=%g outside [2^-20, 2^20]", (double)opt->epsilon);
  if (!(opt->light_fraction >= 0.0f && opt->light_fraction <= 1.0f))
    return fail(CC_EINVAL, "light_fraction=%g outside [0, 1]", (double)opt->light_fraction);
  return CC_OK;
}

template <typename I>
// orig_of (nullable): the CSR's vertices were renumbered; forest edges are
// written in the original numbering.
static cc_status amsf_run(StaticArgs& a, const AmsfLayout& L, const float* w, const cc_amsf_options* opt,
                          AmsfHostBlock* hb_host, int32_t* edges_u, int32_t* edges_v, float* edges_w,
                          int64_t* num_edges, double* weight_dev, const int32_t* orig_of) {
  char* ws = a.ws;
  float* thr = (float*)(ws + L.thr);
  AmsfHostBlock* hb = (AmsfHostBlock*)(ws + L.hostblk);
  AmsfScalars* as = &hb->sc;
  float* hookw = (float*)(ws + L.hookw);
  int32_t* tile_row = (int32_t*)(ws + L.tile_row);
  long long* lpart = (long long*)(ws + L.lpart);
  int2* luv = (int2*)(ws + L.luv);
  float* lw = (float*)(ws + L.lw);
  const int64_t n = a.n, m = a.m;
  const unsigned G = (unsigned)std::min<int64_t>(std::max<int64_t>(L.ntiles, 1), kAmsfPassGrid);
  const int aligned = (((uintptr_t)w | (uintptr_t)a.adj) & 15u) == 0;
  {
    PhaseScope ps(a.ctx, a.s, "init");
    // every parent of the array gets a valid value, also beyond the swept
    // vertices of a restricted call
    const int64_t np = a.n_parents > n ? a.n_parents : n;
    hipLaunchKernelGGL(k_amsf_iota, dim3(grid_for(np, kFBlock, 4096)), dim3(kFBlock), 0, a.s, np, a.P);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(2 * n, kFBlock, 4096)), dim3(kFBlock), 0, a.s, (uint32_t*)a.hook_e,
                       2 * n, 0xffffffffu);
    CC_LAUNCH_CHECK();
  }
  {
    PhaseScope ps(a.ctx, a.s, "amsf_buckets");
    RangePart* part = (RangePart*)(ws + L.range);
    const unsigned gr = grid_for(std::max<int64_t>(div_up(m, 4), 1), kFBlock, kAmsfRangeGrid);
    hipLaunchKernelGGL(k_amsf_range, dim3(gr), dim3(kFBlock), 0, a.s, m, w, (int)(((uintptr_t)w & 15u) == 0), part);
    hipLaunchKernelGGL(k_amsf_setup, dim3(1), dim3(1024), 0, a.s, (const RangePart*)part, (int)gr,
                       (double)opt->epsilon, opt->light_fraction, sm_out(opt->seed, kTagAmsf), m, w, thr, as,
                       hb->shist);
    // every row of the CSR, also beyond the swept vertices of a restricted
    // call: then each tile's first row is right even if rows after the
    // swept ones were not empty, and the pass reads only rows and offsets
    // inside the arrays
    const int64_t nt = a.n_parents > n ? a.n_parents : n;
    hipLaunchKernelGGL(k_amsf_tile_rows<I>, dim3(grid_for(nt, kFBlock, 4096)), dim3(kFBlock), 0, a.s, nt,
                       (const I*)a.off, tile_row);
    hipLaunchKernelGGL((k_amsf_pass<I, false>), dim3(G), dim3(kAmsfThreads), 0, a.s, n, m, (const I*)a.off, a.adj,
                       w, (const float*)thr, (const AmsfScalars*)as, (const int32_t*)tile_row, L.ntiles, -1, lpart,
                       (const long long*)nullptr, (int2*)nullptr, (float*)nullptr, aligned);
    hipLaunchKernelGGL(k_amsf_row_scan, dim3(kAmsfLightMax), dim3(1024), 0, a.s, lpart, (int)G,
                       (const AmsfScalars*)as, hb->rowsum);
    hipLaunchKernelGGL(k_amsf_lstart, dim3(1), dim3(1024), 0, a.s, (const AmsfScalars*)as,
                       (const long long*)hb->rowsum, hb->lstart);
    CC_LAUNCH_CHECK();
    CC_HIP(hipMemcpyAsync(hb_host, hb, sizeof(AmsfHostBlock), hipMemcpyDeviceToHost, a.s));
    CC_HIP(hipStreamSynchronize(a.s));
  }
  const AmsfScalars& hs = hb_host->sc;
  if (hs.bad) return fail(CC_EINVAL, "%u weights are not finite and > 0", hs.bad);
  if (hs.too_many)
    return fail(CC_EINVAL, "weights from %g to %g need more than %d buckets at epsilon=%g", (double)hs.wmin,
                (double)hs.wmax, kAmsfMaxBuckets, (double)opt->epsilon);
  const int nb = hs.nb;
  // light buckets that fit the sorted list
  int b0 = nb > 0 ? hs.b0 : 0;
  while (b0 > 0 && hb_host->lstart[b0] > L.cap) --b0;
  a.sample_rounds = b0;
  {
    PhaseScope ps(a.ctx, a.s, "amsf_light");
    if (b0 > 0) {
      hipLaunchKernelGGL((k_amsf_pass<I, true>), dim3(G), dim3(kAmsfThreads), 0, a.s, n, m, (const I*)a.off, a.adj,
                         w, (const float*)thr, (const AmsfScalars*)as, (const int32_t*)tile_row, L.ntiles, b0, lpart,
                         (const long long*)hb->lstart, luv, lw, aligned);
      int b = 0;
      while (b < b0) {
        const long long c = hb_host->lstart[b + 1] - hb_host->lstart[b];
        if (c > kAmsfSeqMax) {
          hipLaunchKernelGGL(k_amsf_light, dim3(grid_for(c, kFBlock, 8192)), dim3(kFBlock), 0, a.s,
                             (const int2*)luv, (const float*)lw, hb_host->lstart[b], hb_host->lstart[b + 1], a.P,
                             a.hook_e, hookw);
          ++b;
          continue;
        }
        int e = b;
        while (e < b0 && hb_host->lstart[e + 1] - hb_host->lstart[e] <= kAmsfSeqMax) ++e;
        hipLaunchKernelGGL(k_amsf_light_seq, dim3(1), dim3(kAmsfSeqThreads), 0, a.s, (const int2*)luv,
                           (const float*)lw, (const long long*)hb->lstart, b, e, a.P, a.hook_e, hookw);
        b = e;
      }
      CC_LAUNCH_CHECK();
    }
  }
  a.finish_rounds = 0;
  if (b0 < nb) {
    PhaseScope ps(a.ctx, a.s, "amsf_rounds");
    // Candidate lists of the vertices outside L_max, built once; the
    // low-degree list then shrinks round by round as its vertices join
    // L_max, the short lists of higher-degree vertices are kept as built.
    cc_status st = prepare_candidates<I>(a);
    if (st != CC_OK) return st;
    CC_HIP(hipMemcpyAsync(a.ctx->host, a.ctx->dev, sizeof(DevScalars), hipMemcpyDeviceToHost, a.s));
    CC_HIP(hipStreamSynchronize(a.s));
    const DevScalars hsc = *a.ctx->host;
    uint32_t* rcnt = &as->pad[0];
    hipLaunchKernelGGL(k_amsf_round_init, dim3(1), dim3(1), 0, a.s, (const DevScalars*)a.ctx->dev, rcnt);
    const CandLists cl = a.lists();
    const I* offI = (const I*)a.off;
    int32_t* lists[2] = {a.cand, a.count};
    const unsigned gthr = (unsigned)std::max<int64_t>(div_up(hsc.bin_count[0], kAmsfRoundTile), 1);
    for (int b = b0; b < nb; ++b) {
      const int r = b - b0;
      const AmsfRoundOp op{a.P, w, (const float*)thr, b, a.hook_e, hookw};
      if (hsc.bin_count[0] > 0)
        hipLaunchKernelGGL(k_amsf_round<I>, dim3(gthr), dim3(kAmsfRoundThreads), 0, a.s,
                           (const int32_t*)lists[r & 1], lists[(r + 1) & 1], rcnt, r, offI, a.adj, w,
                           (const float*)thr, b, a.P, hsc.lmax, a.hook_e, hookw);
      if (hsc.bin_count[1] > 0)
        hipLaunchKernelGGL((k_visit_wave<AmsfRoundOp, I>), dim3(grid_for((int64_t)hsc.bin_count[1] * kWave, kFBlock, 2048)),
                           dim3(kFBlock), 0, a.s, cl.big, cl.bins, offI, a.adj, op, (uint32_t*)nullptr);
      if (hsc.bin_count[2] > 0)
        hipLaunchKernelGGL((k_visit_block<AmsfRoundOp, I>), dim3(1024), dim3(kFBlock), 0, a.s, cl.n, cl.big, cl.bins,
                           offI, a.adj, op, (uint32_t*)nullptr);
      if (hsc.bin_count[3] > 0)
        hipLaunchKernelGGL((k_visit_heavy<AmsfRoundOp, I>), dim3(2048), dim3(kFBlock), 0, a.s, cl.heavy,
                           &cl.bins[3], cl.hp, offI, a.adj, op, (uint32_t*)nullptr);
      CC_LAUNCH_CHECK();
      ++a.finish_rounds;
    }
  }
  cc_status st = output_labels(a);
  if (st != CC_OK) return st;
  st = forest_filter(a.s, n, nullptr, a.hook_e, hookw, (int32_t*)(ws + L.fcnt), edges_u, edges_v, edges_w,
                     num_edges, orig_of);
  if (st != CC_OK) return st;
  if (weight_dev) {  // edges_w is non-NULL (checked at entry)
    double* wpart = (double*)(ws + L.wpart);
    hipLaunchKernelGGL(k_amsf_weight, dim3(kAmsfWeightGrid), dim3(kFBlock), 0, a.s, (const float*)edges_w,
                       (const long long*)num_edges, wpart);
    hipLaunchKernelGGL(k_amsf_weight_sum, dim3(1), dim3(kFBlock), 0, a.s, (const double*)wpart, kAmsfWeightGrid,
                       weight_dev);
    CC_LAUNCH_CHECK();
  }
  return CC_OK;
}

}  // namespace cc

using namespace cc;

extern "C" {

cc_status cc_amsf_default_options(cc_amsf_options* out) {
  if (!out) return fail(CC_EINVAL, "out is NULL");
  out->epsilon = 0.25f;
  out->light_fraction = 0.4f;
  out->seed = 0x5eedULL;
  return CC_OK;
}

cc_status cc_amsf_workspace_bytes(int64_t n, int64_t m, const cc_amsf_options* opt, size_t* bytes) {
  if (!bytes) return fail(CC_EINVAL, "bytes is NULL");
  cc_status st = check_amsf_options(opt);
  if (st != CC_OK) return st;
  if (n < 1 || n > 0x7fffffffLL) return fail(CC_EINVAL, "n=%lld outside [1, 2^31-1]", (long long)n);
  if (m < 0) return fail(CC_EINVAL, "m < 0");
  *bytes = amsf_layout(n, m, opt->light_fraction).total;
  return CC_OK;
}

cc_status cc_amsf_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                      const int32_t* adj, const float* weights, const cc_amsf_options* opt, void* workspace,
                      size_t ws_bytes, int32_t* labels_out, int32_t* edges_u, int32_t* edges_v, float* edges_w,
                      int64_t* num_edges_dev, double* weight_dev, void* hip_stream) {
  cc_status st = check_amsf_options(opt);
  if (st != CC_OK) return st;
  if (!edges_u || !edges_v || !num_edges_dev) return fail(CC_EINVAL, "NULL forest output");
  if (m > 0 && !weights) return fail(CC_EINVAL, "weights are NULL");
  if (weight_dev && !edges_w) return fail(CC_EINVAL, "weight_dev needs edges_w");
  size_t need = 0;
  st = cc_amsf_workspace_bytes(n, m, opt, &need);
  if (st != CC_OK) return st;
  if (!workspace || ws_bytes < need)
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
  const AmsfLayout L = amsf_layout(n, m, opt->light_fraction);
  const cc_variant v = amsf_variant();
  StaticArgs a;
  st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, &v, workspace, L.hook, labels_out, nullptr,
                  hip_stream);
  if (st != CC_OK) return st;
  a.hook_e = (int2*)((char*)workspace + L.hook);
  if (!ctx->amsf_host) CC_HIP(hipHostMalloc((void**)&ctx->amsf_host, sizeof(AmsfHostBlock), hipHostMallocDefault));
  st = offsets_are_64bit ? amsf_run<int64_t>(a, L, weights, opt, (AmsfHostBlock*)ctx->amsf_host, edges_u, edges_v,
                                             edges_w, num_edges_dev, weight_dev, nullptr)
                         : amsf_run<int32_t>(a, L, weights, opt, (AmsfHostBlock*)ctx->amsf_host, edges_u, edges_v,
                                             edges_w, num_edges_dev, weight_dev, nullptr);
  cc_stats& s = ctx->last;
  s.n = n;
  s.m = m;
  s.sample_rounds = a.sample_rounds;
  s.finish_rounds = a.finish_rounds;
  return st;
}

cc_status cc_amsf_mapped_workspace_bytes(int64_t n, int64_t m, const cc_amsf_options* opt, size_t* bytes) {
  cc_status st = cc_amsf_workspace_bytes(n, m, opt, bytes);
  if (st != CC_OK) return st;
  *bytes += align256((size_t)n * 4);  // the labels in the CSR's numbering
  return CC_OK;
}

cc_status cc_amsf_csr_mapped(cc_ctx* ctx, int64_t n, int64_t n_active, int64_t m, const void* offsets,
                             int offsets_are_64bit, const int32_t* adj, const int32_t* orig_of, const int32_t* new_of,
                             const float* weights, const cc_amsf_options* opt, void* workspace, size_t ws_bytes,
                             int32_t* labels_out, int32_t* edges_u, int32_t* edges_v, float* edges_w,
                             int64_t* num_edges_dev, double* weight_dev, void* hip_stream) {
  cc_status st = check_amsf_options(opt);
  if (st != CC_OK) return st;
  if (!edges_u || !edges_v || !num_edges_dev || !labels_out) return fail(CC_EINVAL, "NULL output");
  if (!orig_of || !new_of) return fail(CC_EINVAL, "NULL permutation argument");
  if (n_active < 0 || n_active > n) return fail(CC_EINVAL, "n_active=%lld outside [0, n]", (long long)n_active);
  if (m > 0 && !weights) return fail(CC_EINVAL, "weights are NULL");
  if (weight_dev && !edges_w) return fail(CC_EINVAL, "weight_dev needs edges_w");
  size_t need = 0;
  st = cc_amsf_mapped_workspace_bytes(n, m, opt, &need);
  if (st != CC_OK) return st;
  if (!workspace || ws_bytes < need)
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
  // the layout of the whole graph; the algorithm runs on the first na
  // vertices (the others have empty rows: alone in their components, no
  // forest edges), with the labels in the CSR's numbering after the layout
  const AmsfLayout L = amsf_layout(n, m, opt->light_fraction);
  const int64_t na = n_active > 0 ? n_active : 1;
  int32_t* Pnew = (int32_t*)((char*)workspace + L.total);
  const cc_variant v = amsf_variant();
  StaticArgs a;
  st = setup_args(a, ctx, na, m, offsets, offsets_are_64bit, adj, &v, workspace, L.hook, Pnew, nullptr, hip_stream);
  if (st != CC_OK) return st;
  a.n_parents = n;
  a.map_orig = orig_of;
  a.map_rmin = a.count;
  a.hook_e = (int2*)((char*)workspace + L.hook);
  if (!ctx->amsf_host) CC_HIP(hipHostMalloc((void**)&ctx->amsf_host, sizeof(AmsfHostBlock), hipHostMallocDefault));
  st = offsets_are_64bit ? amsf_run<int64_t>(a, L, weights, opt, (AmsfHostBlock*)ctx->amsf_host, edges_u, edges_v,
                                             edges_w, num_edges_dev, weight_dev, orig_of)
                         : amsf_run<int32_t>(a, L, weights, opt, (AmsfHostBlock*)ctx->amsf_host, edges_u, edges_v,
                                             edges_w, num_edges_dev, weight_dev, orig_of);
  if (st == CC_OK) st = map_back_labels(a, n, orig_of, new_of, Pnew, labels_out);
  cc_stats& s = ctx->last;
  s.n = n;
  s.m = m;
  s.sample_rounds = a.sample_rounds;
  s.finish_rounds = a.finish_rounds;
  return st;
}

}  // extern "C"
