// Learned variant selector: graph features, a 16 -> 64 -> 64 -> K MLP with
// hand-written forward / backward / Adam kernels, and an automatic static
// entry point that picks a sampling x finish arm per graph.
//
// This part is not in the paper (its only selection guidance is a decision
// tree whose rules are stated in its text: no sampling when m/n < 3, BFS or
// LDD on dense low-diameter graphs, k-out otherwise, UF-Rem-CAS + FindNaive
// to finish).  It changes speed only: every arm returns the same canonical
// labels.
//
// Features (16 FP32), computed on the device in three launches and read back
// with the model's choice in one copy:
//   0 log2 n          1 log2(m+1)         2 m/n               3 degree CV
//   4 max/mean deg    5 frac deg 0        6 frac deg 1        7 frac deg <= 2
//   8 degree skew     14 [m/n < 3]        15 log2(max deg + 1)
// and, over 4096 seeded vertex draws v (those with an edge; f = the first
// entry of v's row):
//   9 mean [f < v]    10 mean log2(1 + |v - f|) / log2(n + 1)
//   11 mean log2(1 + deg f)
// and 16 BFS probes from seeded sources, each expanding whole levels while
// at most 1024 adjacency entries are scanned and at most 4 levels:
//   12 mean levels expanded     13 mean vertices reached / n
//
// MLP: parameters packed as BF16 [W1 16x64 | b1 64 | W2 64x64 | b2 64 |
// W3 64xK | b3 K] (row-major, input index first).  Inputs and hidden
// activations are rounded to BF16; every product is accumulated in FP32;
// outputs are FP32 predicted log-time ratios; ReLU between layers.  The
// backward pass treats the BF16 rounding as identity (straight-through) and
// the ReLU derivative at 0 as 0.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "cc_frontier.h"
#include "cc_static.h"

namespace cc {

constexpr int kIn = 16, kH = 64;
constexpr int kMaxArms = 128;

__host__ __device__ inline int64_t mlp_param_count(int K) { return (int64_t)kIn * kH + kH + kH * kH + kH + kH * K + K; }

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
// Round-to-nearest-even FP32 -> BF16 (finite inputs).
__host__ __device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_round(float f) { return bf16_to_f32(f32_to_bf16(f)); }

struct MlpView {
  const uint16_t *W1, *b1, *W2, *b2, *W3, *b3;
};
__device__ __forceinline__ MlpView mlp_view(const uint16_t* p, int K) {
  MlpView v;
  v.W1 = p;
  v.b1 = v.W1 + kIn * kH;
  v.W2 = v.b1 + kH;
  v.b2 = v.W2 + kH * kH;
  v.W3 = v.b2 + kH;
  v.b3 = v.W3 + kH * K;
  return v;
}

// One row of the forward pass by a block of at least kH threads (thread t
// computes hidden unit t): xin (FP32, kIn values) -> Y (K values).  cache
// (nullable): [z1 64 | a1 64 | z2 64 | a2 64].
__device__ __forceinline__ void mlp_forward_row(const MlpView& P, int K, const float* xin, float* x, float* a1,
                                                float* a2, float* Y, float* cache) {
  const int t = threadIdx.x;
  if (t < kIn) x[t] = bf16_round(xin[t]);
  __syncthreads();
  if (t < kH) {
    float z = bf16_to_f32(P.b1[t]);
    for (int i = 0; i < kIn; ++i) z += x[i] * bf16_to_f32(P.W1[i * kH + t]);
    const float h1 = bf16_round(z > 0.f ? z : 0.f);
    a1[t] = h1;
    if (cache) {
      cache[t] = z;
      cache[kH + t] = h1;
    }
  }
  __syncthreads();
  if (t < kH) {
    float z = bf16_to_f32(P.b2[t]);
    for (int i = 0; i < kH; ++i) z += a1[i] * bf16_to_f32(P.W2[i * kH + t]);
    const float h2 = bf16_round(z > 0.f ? z : 0.f);
    a2[t] = h2;
    if (cache) {
      cache[2 * kH + t] = z;
      cache[3 * kH + t] = h2;
    }
  }
  __syncthreads();
  for (int j = t; j < K; j += blockDim.x) {
    float y = bf16_to_f32(P.b3[j]);
    for (int i = 0; i < kH; ++i) y += a2[i] * bf16_to_f32(P.W3[i * K + j]);
    Y[j] = y;
  }
}

// The forward pass and argmin of one feature row with a block of 4 * kH
// threads: four lanes per unit, each summing a quarter of the unit's inputs,
// combined with two shuffles; the argmin is one wave reduction that keeps
// the smallest index among equal minima, as a scan in index order does.
// (One lane per unit, as in mlp_forward_row, costs 64 dependent steps per
// layer: 2.2 us of the decision kernel's 11.)
__device__ __forceinline__ float quad_sum(float z) {
  z += __shfl_xor(z, 1, kWave);
  return z + __shfl_xor(z, 2, kWave);
}

__device__ void decide_row(const MlpView& P, int K, const float* xin, float* x, float* a1, float* a2, float* Y,
                           int32_t* chosen) {
  const int t = threadIdx.x, u = t >> 2, q = t & 3;
  if (t < kIn) x[t] = bf16_round(xin[t]);
  __syncthreads();
  {
    float z = 0.f;
#pragma unroll
    for (int i = 4 * q; i < 4 * q + 4; ++i) z += x[i] * bf16_to_f32(P.W1[i * kH + u]);
    z = quad_sum(z) + bf16_to_f32(P.b1[u]);
    if (q == 0) a1[u] = bf16_round(z > 0.f ? z : 0.f);
  }
  __syncthreads();
  {
    float z = 0.f;
#pragma unroll
    for (int i = 16 * q; i < 16 * q + 16; ++i) z += a1[i] * bf16_to_f32(P.W2[i * kH + u]);
    z = quad_sum(z) + bf16_to_f32(P.b2[u]);
    if (q == 0) a2[u] = bf16_round(z > 0.f ? z : 0.f);
  }
  __syncthreads();
  for (int base = 0; base < K; base += kH) {
    const int j = base + u < K ? base + u : K - 1;   // a whole quad takes the same output
    float y = 0.f;
#pragma unroll
    for (int i = 16 * q; i < 16 * q + 16; ++i) y += a2[i] * bf16_to_f32(P.W3[i * K + j]);
    y = quad_sum(y) + bf16_to_f32(P.b3[j]);
    if (q == 0 && base + u < K) Y[j] = y;
  }
  __syncthreads();
  if (t < kWave) {
    float v = t < K ? Y[t] : INFINITY;
    int c = t;
    for (int j = t + kWave; j < K; j += kWave)
      if (Y[j] < v) v = Y[j], c = j;
    for (int o = 32; o > 0; o >>= 1) {
      const float v2 = __shfl_xor(v, o, kWave);
      const int c2 = __shfl_xor(c, o, kWave);
      if (v2 < v || (v2 == v && c2 < c)) v = v2, c = c2;
    }
    if (t == 0) *chosen = c;
  }
}

// One block per row.
__global__ void __launch_bounds__(kH) k_mlp_forward(const uint16_t* __restrict__ params, int K, int B,
                                                    const float* __restrict__ X, float* __restrict__ Y,
                                                    float* __restrict__ cache) {
  __shared__ float x[kIn], a1[kH], a2[kH];
  const int r = blockIdx.x;
  if (r >= B) return;
  mlp_forward_row(mlp_view(params, K), K, X + (int64_t)r * kIn, x, a1, a2, Y + (int64_t)r * K,
                  cache ? cache + (int64_t)r * 4 * kH : nullptr);
}

// Gradients of the mean squared error L = mean_{r,j} (Y - T)^2 with respect
// to every parameter (FP32, same packing as the parameters).  One block;
// scratch holds 4 * B * 64 floats.  loss (nullable) receives L.
__global__ void __launch_bounds__(256) k_mlp_backward(const uint16_t* __restrict__ params, int K, int B,
                                                      const float* __restrict__ X, const float* __restrict__ cache,
                                                      const float* __restrict__ Y, const float* __restrict__ T,
                                                      float* __restrict__ grads, float* __restrict__ scratch,
                                                      float* loss) {
  const MlpView P = mlp_view(params, K);
  const int t = threadIdx.x, nt = blockDim.x;
  float* dY = scratch;                        // B x K (K <= 128 = 2*64)
  float* dZ2 = scratch + (int64_t)B * 2 * kH;  // B x 64
  float* dZ1 = dZ2 + (int64_t)B * kH;         // B x 64
  const float scale = 2.0f / (float)((int64_t)B * K);
  __shared__ float red[256];
  float ls = 0.f;
  for (int64_t e = t; e < (int64_t)B * K; e += nt) {
    const float d = Y[e] - T[e];
    dY[e] = scale * d;
    ls += d * d;
  }
  red[t] = ls;
  __syncthreads();
  if (t == 0) {
    float s = 0.f;
    for (int i = 0; i < nt; ++i) s += red[i];
    if (loss) *loss = s / (float)((int64_t)B * K);
  }
  float* gW1 = grads;
  float* gb1 = gW1 + kIn * kH;
  float* gW2 = gb1 + kH;
  float* gb2 = gW2 + kH * kH;
  float* gW3 = gb2 + kH;
  float* gb3 = gW3 + kH * K;
  __syncthreads();
  // layer 3
  for (int e = t; e < kH * K; e += nt) {
    const int i = e / K, j = e % K;
    float s = 0.f;
    for (int r = 0; r < B; ++r) s += cache[(int64_t)r * 4 * kH + 3 * kH + i] * dY[(int64_t)r * K + j];
    gW3[e] = s;
  }
  for (int j = t; j < K; j += nt) {
    float s = 0.f;
    for (int r = 0; r < B; ++r) s += dY[(int64_t)r * K + j];
    gb3[j] = s;
  }
  for (int64_t e = t; e < (int64_t)B * kH; e += nt) {
    const int r = (int)(e / kH), i = (int)(e % kH);
    float s = 0.f;
    for (int j = 0; j < K; ++j) s += dY[(int64_t)r * K + j] * bf16_to_f32(P.W3[i * K + j]);
    dZ2[e] = cache[(int64_t)r * 4 * kH + 2 * kH + i] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // layer 2
  for (int e = t; e < kH * kH; e += nt) {
    const int i = e / kH, j = e % kH;
    float s = 0.f;
    for (int r = 0; r < B; ++r) s += cache[(int64_t)r * 4 * kH + kH + i] * dZ2[(int64_t)r * kH + j];
    gW2[e] = s;
  }
  for (int j = t; j < kH; j += nt) {
    float s = 0.f;
    for (int r = 0; r < B; ++r) s += dZ2[(int64_t)r * kH + j];
    gb2[j] = s;
  }
  for (int64_t e = t; e < (int64_t)B * kH; e += nt) {
    const int r = (int)(e / kH), i = (int)(e % kH);
    float s = 0.f;
    for (int j = 0; j < kH; ++j) s += dZ2[(int64_t)r * kH + j] * bf16_to_f32(P.W2[i * kH + j]);
    dZ1[e] = cache[(int64_t)r * 4 * kH + i] > 0.f ? s : 0.f;
  }
  __syncthreads();
  // layer 1
  for (int e = t; e < kIn * kH; e += nt) {
    const int i = e / kH, j = e % kH;
    float s = 0.f;
    for (int r = 0; r < B; ++r) s += bf16_round(X[(int64_t)r * kIn + i]) * dZ1[(int64_t)r * kH + j];
    gW1[e] = s;
  }
  for (int j = t; j < kH; j += nt) {
    float s = 0.f;
    for (int r = 0; r < B; ++r) s += dZ1[(int64_t)r * kH + j];
    gb1[j] = s;
  }
}

// Adam on FP32 master weights; the BF16 parameters are refreshed from them.
__global__ void k_mlp_adam(float* __restrict__ master, uint16_t* __restrict__ params, const float* __restrict__ g,
                           float* __restrict__ m1, float* __restrict__ m2, int64_t count, float lr, float b1,
                           float b2, float eps, float bc1, float bc2) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) {
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float c = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = c;
    const float w = master[i] - lr * (a / bc1) / (sqrtf(c / bc2) + eps);
    master[i] = w;
    params[i] = f32_to_bf16(w);
  }
}

__global__ void k_f32_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = f32_to_bf16(src[i]);
}

// ---- feature kernels ----------------------------------------------------------
//
// Two launches compute everything: in the first, blocks [0, nb) sweep the
// degrees and the vertex draws into per-block partials and blocks nb ..
// nb + kProbes - 1 run one budgeted BFS each; the second (one block)
// reduces the partials, forms the 16 features, normalises them, runs the
// forward pass, picks the arm and writes the 17 words straight into the
// context's pinned host buffer; the host synchronises once.

// Pass blocks: few enough that the one-block decision kernel's reduction of
// their partials stays short (1024 blocks cost about 4 us more per call on
// graphs of 2^22 vertices than 256 do, the sweep itself included).
constexpr int kFeatBlocks = 256;
constexpr int kFeatThreads = 256;
constexpr int kFeatSamples = 4096;
constexpr int kProbeLevels = 4;
constexpr int kProbeEdges = 1024;
constexpr int kProbeSlots = 2048;     // LDS hash of discovered vertices: load <= 1/2
constexpr int kProbeCap = kProbeEdges + 1;   // frontier capacity (a level discovers <= kProbeEdges)
constexpr int kProbes = 16;           // independent probes from seeded sources, one block each
constexpr int kPart = 12;             // doubles per block of partial sums
constexpr uint64_t kTagFeat = 0x66656174ULL;  // "feat"

// Selector area of the workspace: probe results; the per-block
// partials (at most n/1024 + 1 blocks of 96 bytes) use the n-int count area.
constexpr size_t kSelProbe = 0;                // kProbes x [levels, reached]

// Dynamic roles share one LDS buffer.
constexpr size_t kProbeSmem = 2 * (size_t)kProbeCap * 8 + (size_t)kProbeSlots * 4 + 4 * (size_t)kProbeCap * 4 +
                               (size_t)(kProbeCap + 1) * 4 + 64;
constexpr size_t kFinishSmem = (size_t)kPart * kFeatThreads * 8 + (3 * kIn + 2 * kH + kMaxArms) * 4 + 16;
constexpr size_t kFeatSmem = kProbeSmem;

struct NormArg {
  float v[2 * kIn];   // mean[16], sd[16]
};

__device__ __forceinline__ double max_d(double a, double b) { return b > a ? b : a; }
__device__ __forceinline__ double combine(int k, double a, double b) { return k == 3 ? max_d(a, b) : a + b; }

// Partials of one pass block: [sum d, sum d^2, sum d^3, max d, #d==0,
// #d==1, #d<=2, #draws with an edge, #(f < v), sum locality,
// sum log2(1 + deg f), 0].
template <typename I>
__device__ void feat_pass(int64_t n, const I* __restrict__ off, const int32_t* __restrict__ adj, uint64_t key,
                          int nb, double* __restrict__ part, double* red) {
  double q[kPart] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int64_t stride = (int64_t)nb * kFeatThreads;
  const int64_t gid = blockIdx.x * (int64_t)kFeatThreads + threadIdx.x;
  // four vertices per lane: five row bounds loaded together
  for (int64_t v0 = 4 * gid; v0 < n; v0 += 4 * stride) {
    int64_t o[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) o[j] = v0 + j <= n ? (int64_t)off[v0 + j] : 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (v0 + j >= n) break;
      const double d = (double)(o[j + 1] - o[j]);
      q[0] += d;
      q[1] += d * d;
      q[2] += d * d * d;
      q[3] = max_d(q[3], d);
      q[4] += d == 0.0;
      q[5] += d == 1.0;
      q[6] += d <= 2.0;
    }
  }
  const double ln = log2((double)n + 1.0);
  for (int64_t i = gid; i < kFeatSamples; i += stride) {
    const int64_t v = (int64_t)(sm_out(key, (uint64_t)i) % (uint64_t)n);
    const int64_t b = (int64_t)off[v];
    if ((int64_t)off[v + 1] == b) continue;
    const int64_t f = adj[b];
    q[7] += 1.0;
    q[8] += f < v;
    q[9] += log2(1.0 + (double)(v > f ? v - f : f - v)) / ln;
    q[10] += log2(1.0 + (double)((int64_t)off[f + 1] - (int64_t)off[f]));
  }
  constexpr int kW = kFeatThreads / kWave;
  for (int k = 0; k < kPart; ++k) {
    double x = q[k];
    for (int o = 32; o > 0; o >>= 1) x = combine(k, x, __shfl_xor(x, o, kWave));
    if (lane_id() == 0) red[k * kW + threadIdx.x / kWave] = x;
  }
  __syncthreads();
  if (threadIdx.x < kPart) {
    const int k = threadIdx.x;
    double x = red[k * kW];
    for (int w = 1; w < kW; ++w) x = combine(k, x, red[k * kW + w]);
    part[(int64_t)k * nb + blockIdx.x] = x;  // one row per partial, so the final reads coalesce
  }
}

// Whole-level BFS within an edge budget, entirely in LDS: a hash table of
// discovered vertices and two frontier queues holding each vertex's row
// start and degree (loaded once, when the vertex is discovered).  Before a
// level is expanded its frontier's degrees are summed and the search stops
// if the budget would be exceeded, so which vertices are reached does not
// depend on scheduling.  out: [levels, reached].
template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T* wtot, T* total) {
  constexpr int kW = kFeatThreads / kWave;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  T inc = x;
  for (int o = 1; o < kWave; o <<= 1) {
    const T y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) wtot[w] = inc;
  __syncthreads();
  T before = 0, all = 0;
  for (int i = 0; i < kW; ++i) {
    if (i < w) before += wtot[i];
    all += wtot[i];
  }
  if (threadIdx.x == 0) *total = all;
  __syncthreads();
  return before + inc - x;
}

template <typename I>
__device__ void feat_probe(const I* __restrict__ off, const int32_t* __restrict__ adj, int32_t src,
                           int64_t* __restrict__ out, unsigned char* smem) {
  int64_t* qst = (int64_t*)smem;                           // [2][kProbeCap] row starts
  int32_t* slots = (int32_t*)(qst + 2 * kProbeCap);        // hash of discovered vertices
  int32_t* qid = slots + kProbeSlots;                      // [2][kProbeCap] vertex ids
  int32_t* qdg = qid + 2 * kProbeCap;                      // [2][kProbeCap] degrees (clamped)
  int32_t* pre = qdg + 2 * kProbeCap;                      // [kProbeCap + 1] frontier degree prefix
  long long* wtot = (long long*)(((uintptr_t)(pre + kProbeCap + 1) + 7) & ~(uintptr_t)7);
  long long* total = wtot + kFeatThreads / kWave;
  int32_t* nnext = (int32_t*)(total + 1);
  const int t = threadIdx.x;
  for (int i = t; i < kProbeSlots; i += kFeatThreads) slots[i] = -1;
  __syncthreads();
  auto insert = [&](int32_t w) -> bool {
    uint32_t h = ((uint32_t)w * 2654435761u) & (kProbeSlots - 1);
    while (true) {
      const int32_t prev = atomicCAS(&slots[h], -1, w);
      if (prev == -1) return true;
      if (prev == w) return false;
      h = (h + 1) & (kProbeSlots - 1);
    }
  };
  auto push = [&](int q, int32_t pos, int32_t w) {
    const int64_t b = (int64_t)off[w], d = (int64_t)off[w + 1] - b;
    qid[q * kProbeCap + pos] = w;
    qst[q * kProbeCap + pos] = b;
    qdg[q * kProbeCap + pos] = (int32_t)(d < kProbeEdges + 1 ? d : kProbeEdges + 1);
  };
  if (t == 0) {
    insert(src);
    push(0, 0, src);
  }
  int cur = 0;
  int32_t f = 1;
  int64_t reached = 1, scanned = 0;
  int levels = 0;
  __syncthreads();
  while (f > 0 && levels < kProbeLevels) {
    // contiguous chunk of the frontier per thread; scan of the chunk sums
    const int32_t chunk = (f + kFeatThreads - 1) / kFeatThreads;
    const int32_t i0 = t * chunk < f ? t * chunk : f;
    const int32_t i1 = i0 + chunk < f ? i0 + chunk : f;
    long long sum = 0;
    for (int32_t i = i0; i < i1; ++i) sum += qdg[cur * kProbeCap + i];
    const long long before = block_excl_scan<long long>(sum, wtot, total);
    const long long fe = *total;
    if (scanned + fe > kProbeEdges) break;
    {
      int32_t acc = (int32_t)before;
      for (int32_t i = i0; i < i1; ++i) {
        pre[i] = acc;
        acc += qdg[cur * kProbeCap + i];
      }
      if (t == 0) {
        pre[f] = (int32_t)fe;
        *nnext = 0;
      }
    }
    __syncthreads();
    const int nq = cur ^ 1;
    for (int32_t e = t; e < (int32_t)fe; e += kFeatThreads) {
      int32_t lo = 0, hi = f - 1;   // owner: largest i with pre[i] <= e
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      const int32_t w = adj[qst[cur * kProbeCap + lo] + (e - pre[lo])];
      if (insert(w)) push(nq, atomicAdd(nnext, 1), w);
    }
    __syncthreads();
    scanned += fe;
    ++levels;
    f = *nnext;
    reached += f;
    cur = nq;
    __syncthreads();
  }
  if (t == 0) {
    out[0] = levels;
    out[1] = reached;
  }
}

// Reduces the partials into the 16 features (out[0..15]).  With a model,
// normalises them, runs the forward pass and writes the argmin arm (smallest
// index on ties) to out[16] as an int32, else -1.
__device__ void feat_finish(int64_t n, int64_t m, const double* part, int nb, const int64_t* probe,
                            const uint16_t* __restrict__ params, int K, const NormArg& norm, float* __restrict__ out,
                            unsigned char* smem) {
  double* red = (double*)smem;                        // [kPart][kFeatThreads]
  float* feat = (float*)(red + kPart * kFeatThreads);
  float* xin = feat + kIn;
  float* x = xin + kIn;
  float* a1 = x + kIn;
  float* a2 = a1 + kH;
  float* Y = a2 + kH;
  const int t = threadIdx.x;
  double q[kPart] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  static_assert(kFeatBlocks <= 4 * kFeatThreads, "four partial rows per thread");
  static_assert(kFeatThreads == 4 * kH, "decide_row takes four lanes per unit");
  {
    double x[4][kPart];   // every load in flight before any is used
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int b = t + j * kFeatThreads;
#pragma unroll
      for (int k = 0; k < kPart; ++k) x[j][k] = b < nb ? part[(int64_t)k * nb + b] : 0.0;   // 0 is neutral for sums and maxima of counts
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int k = 0; k < kPart; ++k) q[k] = combine(k, q[k], x[j][k]);
  }
  // wave shuffles, then the four wave results (an LDS halving tree cost
  // eight synchronised steps)
  constexpr int kW = kFeatThreads / kWave;
  for (int k = 0; k < kPart; ++k) {
    double y = q[k];
    for (int o = 32; o > 0; o >>= 1) y = combine(k, y, __shfl_xor(y, o, kWave));
    if (lane_id() == 0) red[k * kW + t / kWave] = y;
  }
  __syncthreads();
  if (t == 0) {
    double r[kPart];
    for (int k = 0; k < kPart; ++k) {
      r[k] = red[k * kW];
      for (int w = 1; w < kW; ++w) r[k] = combine(k, r[k], red[k * kW + w]);
    }
    double levels = 0, reached = 0;
    for (int p = 0; p < kProbes; ++p) {
      levels += (double)probe[2 * p];
      reached += (double)probe[2 * p + 1];
    }
    levels /= kProbes;
    reached /= kProbes;
    const double dn = (double)n, dm = (double)m;
    const double mean = r[0] / dn;
    const double var = r[1] / dn - mean * mean > 0 ? r[1] / dn - mean * mean : 0.0;
    const double sd = sqrt(var);
    const double skew = sd > 0 ? (r[2] / dn - 3 * mean * var - mean * mean * mean) / (sd * sd * sd) : 0.0;
    const double cnt = r[7];
    feat[0] = (float)log2(dn);
    feat[1] = (float)log2(dm + 1.0);
    feat[2] = (float)(dm / dn);
    feat[3] = (float)(mean > 0 ? sd / mean : 0.0);
    feat[4] = (float)(mean > 0 ? r[3] / mean : 0.0);
    feat[5] = (float)(r[4] / dn);
    feat[6] = (float)(r[5] / dn);
    feat[7] = (float)(r[6] / dn);
    feat[8] = (float)(skew > 1e6 ? 1e6 : skew);
    feat[9] = (float)(cnt > 0 ? r[8] / cnt : 0.0);
    feat[10] = (float)(cnt > 0 ? r[9] / cnt : 0.0);
    feat[11] = (float)(cnt > 0 ? r[10] / cnt : 0.0);
    feat[12] = (float)levels;
    feat[13] = (float)(reached / dn);
    feat[14] = (float)(dm / dn < 3.0 ? 1.0 : 0.0);
    feat[15] = (float)log2(r[3] + 1.0);
    for (int i = 0; i < kIn; ++i) out[i] = feat[i];
  }
  __syncthreads();
  if (!params) {
    if (t == 0) ((int32_t*)out)[kIn] = -1;
    return;
  }
  if (t < kIn) xin[t] = (feat[t] - norm.v[t]) / (norm.v[kIn + t] > 0.f ? norm.v[kIn + t] : 1.f);
  __syncthreads();
  decide_row(mlp_view(params, K), K, xin, x, a1, a2, Y, (int32_t*)out + kIn);
}

template <typename I>
__global__ void __launch_bounds__(kFeatThreads) k_features(int64_t n, const I* __restrict__ off,
                                                           const int32_t* __restrict__ adj, uint64_t key,
                                                           double* part, int64_t* probe, int nb) {
  __shared__ __align__(16) unsigned char smem[kFeatSmem];
  if (blockIdx.x < (unsigned)nb) {
    feat_pass<I>(n, off, adj, key, nb, part, (double*)smem);
  } else {
    const int p = (int)blockIdx.x - nb;
    const int32_t src = (int32_t)(sm_out(key, (uint64_t)(kFeatSamples + p)) % (uint64_t)n);
    feat_probe<I>(off, adj, src, probe + 2 * p, smem);
  }
}

// One block: the model's parameters are first staged in LDS (coalesced), so
// the forward pass reads no global memory.
constexpr int kMaxParams = kIn * kH + kH + kH * kH + kH + kH * kMaxArms + kMaxArms;

__global__ void __launch_bounds__(kFeatThreads) k_feat_final(int64_t n, int64_t m, const double* part, int nb,
                                                             const int64_t* probe, const uint16_t* __restrict__ params,
                                                             int K, NormArg norm, float* __restrict__ out,
                                                             uint32_t seq) {
  __shared__ __align__(16) unsigned char smem[kFinishSmem];
  __shared__ __align__(16) uint16_t lparams[kMaxParams];
  const uint16_t* pp = nullptr;
  if (params) {
    const int64_t cnt = mlp_param_count(K);
    for (int64_t i = threadIdx.x; i < cnt; i += kFeatThreads) lparams[i] = params[i];
    pp = lparams;
  }
  __syncthreads();
  feat_finish(n, m, part, nb, probe, pp, K, norm, out, smem);
  // publish: the 17 result words, then (system scope) the call's sequence
  // number, which the host polls
  __syncthreads();
  if (threadIdx.x == 0)  // thread 0 wrote the words; its system-scope release orders them first
    __hip_atomic_store((uint32_t*)out + kIn + 1, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Features and, with a model, the chosen arm; one host synchronisation.
// `pre` (nullable) is enqueued after the selector's kernels and before the
// host waits for their answer, so that its device work overlaps the wait.
template <typename I>
static cc_status features_impl(StaticArgs& a, const uint16_t* params, int K, const float* norm_host, float* feat,
                               int* chosen, StaticArgs* pre) {
  char* sel = a.ws + a.L.mlp;
  double* part = (double*)(a.ws + a.L.count);
  int64_t* probe = (int64_t*)(sel + kSelProbe);
  const uint64_t key = sm_out(a.v->seed, kTagFeat);
  const int nb = (int)grid_for(div_up(a.n, 4), kFeatThreads, kFeatBlocks);
  NormArg na;
  for (int i = 0; i < 2 * kIn; ++i) na.v[i] = params ? norm_host[i] : 0.f;
  hipLaunchKernelGGL(k_features<I>, dim3(nb + kProbes), dim3(kFeatThreads), 0, a.s, a.n, (const I*)a.off, a.adj, key,
                     part, probe, nb);
  const uint32_t seq = ++a.ctx->sel_seq;
  hipLaunchKernelGGL(k_feat_final, dim3(1), dim3(kFeatThreads), 0, a.s, a.n, a.m, (const double*)part, nb,
                     (const int64_t*)probe, params, K, na, a.ctx->sel_dev, seq);
  CC_LAUNCH_CHECK();
  if (pre) {
    cc_status st = static_init(*pre);
    if (st != CC_OK) return st;
  }
  // The final kernel writes straight into pinned host memory and then the
  // sequence number: poll for it (it arrives microseconds before a stream
  // synchronisation would return); after 50 ms fall back to synchronising,
  // which also reports a failed launch.
  float* h = a.ctx->sel_host;
  volatile uint32_t* flag = (volatile uint32_t*)h + kIn + 1;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 0; __atomic_load_n(flag, __ATOMIC_ACQUIRE) != seq; ++spin) {
    if ((spin & 1023u) == 0 &&
        std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(50)) {
      CC_HIP(hipStreamSynchronize(a.s));
      if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) != seq) return fail(CC_EDEVICE, "selector kernel did not report");
      break;
    }
  }
  memcpy(feat, h, kIn * sizeof(float));
  int32_t c;
  memcpy(&c, &h[kIn], sizeof(c));
  *chosen = c;
  return CC_OK;
}

static cc_status features(StaticArgs& a, const uint16_t* params, int K, const float* norm_host, float* feat,
                          int* chosen, StaticArgs* pre = nullptr) {
  return a.o64 ? features_impl<int64_t>(a, params, K, norm_host, feat, chosen, pre)
               : features_impl<int32_t>(a, params, K, norm_host, feat, chosen, pre);
}

}  // namespace cc

using namespace cc;

extern "C" {

int64_t cc_mlp_param_count(int32_t num_arms) {
  return (num_arms < 1 || num_arms > kMaxArms) ? -1 : mlp_param_count(num_arms);
}

cc_status cc_mlp_forward(const uint16_t* params, int32_t K, int32_t B, const float* X, float* Y, float* cache,
                         void* hip_stream) {
  if (!params || !X || !Y) return fail(CC_EINVAL, "NULL argument");
  if (K < 1 || K > kMaxArms || B < 1) return fail(CC_EINVAL, "bad K or B");
  hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(kH), 0, (hipStream_t)hip_stream, params, K, B, X, Y, cache);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

cc_status cc_mlp_backward(const uint16_t* params, int32_t K, int32_t B, const float* X, const float* cache,
                          const float* Y, const float* T, float* grads, float* scratch, float* loss,
                          void* hip_stream) {
  if (!params || !X || !cache || !Y || !T || !grads || !scratch) return fail(CC_EINVAL, "NULL argument");
  if (K < 1 || K > kMaxArms || B < 1) return fail(CC_EINVAL, "bad K or B");
  hipLaunchKernelGGL(k_mlp_backward, dim3(1), dim3(256), 0, (hipStream_t)hip_stream, params, K, B, X, cache, Y, T,
                     grads, scratch, loss);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

cc_status cc_mlp_adam(float* master, uint16_t* params, const float* grads, float* m1, float* m2, int64_t count,
                      float lr, float beta1, float beta2, float eps, int32_t step, void* hip_stream) {
  if (!master || !params || !grads || !m1 || !m2 || count < 1 || step < 1) return fail(CC_EINVAL, "bad argument");
  const float bc1 = 1.f - std::pow(beta1, (float)step), bc2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3(grid_for(count, 256, 64)), dim3(256), 0, (hipStream_t)hip_stream, master,
                     params, grads, m1, m2, count, lr, beta1, beta2, eps, bc1, bc2);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

cc_status cc_mlp_pack_bf16(const float* src, uint16_t* dst, int64_t count, void* hip_stream) {
  if (!src || !dst || count < 0) return fail(CC_EINVAL, "bad argument");
  if (count == 0) return CC_OK;
  hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid_for(count, 256, 64)), dim3(256), 0, (hipStream_t)hip_stream, src, dst,
                     count);
  CC_LAUNCH_CHECK();
  return CC_OK;
}

cc_status cc_graph_features(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                            const int32_t* adj, void* workspace, size_t ws_bytes, float* features_host,
                            void* hip_stream) {
  if (!features_host) return fail(CC_EINVAL, "features_host is NULL");
  cc_variant v;
  cc_default_variant(&v);
  StaticArgs a;
  // the features never touch the label array: any non-null pointer will do
  cc_status st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, &v, workspace, ws_bytes,
                            (int32_t*)workspace, nullptr, hip_stream);
  if (st != CC_OK) return st;
  int chosen;
  return features(a, nullptr, 0, nullptr, features_host, &chosen);
}

}  // extern "C"

static cc_status check_selector_args(int64_t n, int64_t m, const uint16_t* params_dev, int32_t K,
                                     const cc_variant* arms, const float* norm_host, const cc_variant* def,
                                     size_t ws_bytes, const void* workspace) {
  if (params_dev && (K < 1 || K > kMaxArms || !arms || !norm_host)) return fail(CC_EINVAL, "bad selector arguments");
  if (params_dev)
    for (int j = 0; j < K; ++j) {
      cc_status s2 = check_variant(&arms[j], false);
      if (s2 != CC_OK) return s2;
    }
  // the workspace must serve every arm
  size_t need = ws_layout(n, m, def).total;
  if (params_dev)
    for (int j = 0; j < K; ++j) need = std::max(need, ws_layout(n, m, &arms[j]).total);
  if (!workspace || ws_bytes < need)
    return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
  return CC_OK;
}

// Features, then (with a model) the arm of smallest predicted log-time;
// without a model the default variant and chosen = -1.
static cc_status select_arm(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int o64, const int32_t* adj,
                            const uint16_t* params_dev, int32_t K, const cc_variant* arms, const float* norm_host,
                            void* workspace, size_t ws_bytes, void* hip_stream, float* feat, int* chosen,
                            cc_variant* use, StaticArgs* pre = nullptr) {
  cc_variant def;
  cc_default_variant(&def);
  cc_status st = check_selector_args(n, m, params_dev, K, arms, norm_host, &def, ws_bytes, workspace);
  if (st != CC_OK) return st;
  StaticArgs a;
  st = setup_args(a, ctx, n, m, offsets, o64, adj, &def, workspace, ws_bytes, (int32_t*)workspace, nullptr,
                  hip_stream);
  if (st != CC_OK) return st;
  st = features(a, params_dev, params_dev ? K : 0, norm_host, feat, chosen, pre);
  if (st != CC_OK) return st;
  if (!params_dev) *chosen = -1;
  if (*chosen < -1 || *chosen >= K) return fail(CC_EDEVICE, "selector returned arm %d of %d", *chosen, K);
  *use = *chosen < 0 ? def : arms[*chosen];
  return CC_OK;
}

extern "C" {

cc_status cc_select_variant(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                            const int32_t* adj, const uint16_t* params_dev, int32_t K, const cc_variant* arms,
                            const float* norm_host, void* workspace, size_t ws_bytes, cc_variant* out_host,
                            int32_t* chosen_host, float* features_host, void* hip_stream) {
  if (!out_host) return fail(CC_EINVAL, "out_host is NULL");
  float feat[kIn];
  int chosen;
  cc_status st = select_arm(ctx, n, m, offsets, offsets_are_64bit, adj, params_dev, K, arms, norm_host, workspace,
                            ws_bytes, hip_stream, feat, &chosen, out_host);
  if (st != CC_OK) return st;
  if (chosen_host) *chosen_host = chosen;
  if (features_host) memcpy(features_host, feat, sizeof(feat));
  return CC_OK;
}

cc_status cc_ctx_set_selector_gate(cc_ctx* ctx, int64_t min_vertices, int32_t arm) {
  if (!ctx || min_vertices < 0 || (min_vertices > 0 && arm < 0)) return fail(CC_EINVAL, "bad gate");
  ctx->gate_vertices = min_vertices;
  ctx->gate_arm = min_vertices > 0 ? arm : -1;
  return CC_OK;
}

cc_status cc_connectivity_auto(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                               const int32_t* adj, const uint16_t* params_dev, int32_t K, const cc_variant* arms,
                               const float* norm_host, void* workspace, size_t ws_bytes, int32_t* labels_out,
                               int64_t* num_components_dev, int32_t* chosen_host, float* features_host,
                               void* hip_stream) {
  if (!labels_out) return fail(CC_EINVAL, "labels_out is NULL");
  if (!ctx) return fail(CC_EINVAL, "ctx is NULL");
  float feat[kIn];
  int chosen;
  cc_variant use, def;
  cc_default_variant(&def);
  if (params_dev && ctx->gate_vertices > 0 && n < ctx->gate_vertices) {
    // below the gate the model's fixed cost exceeds what it saves: run the
    // gate's arm without features
    if (ctx->gate_arm >= K) return fail(CC_EINVAL, "gate arm %d of %d", ctx->gate_arm, K);
    cc_status st = check_selector_args(n, m, params_dev, K, arms, norm_host, &def, ws_bytes, workspace);
    if (st != CC_OK) return st;
    if (chosen_host) *chosen_host = ctx->gate_arm;
    if (features_host)
      for (int i = 0; i < kIn; ++i) features_host[i] = NAN;
    StaticArgs a;
    st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, &arms[ctx->gate_arm], workspace, ws_bytes,
                    labels_out, num_components_dev, hip_stream);
    if (st != CC_OK) return st;
    return static_run(a);
  }
  // Algorithm 1's init is the same for every arm: it is enqueued behind the
  // selector's kernels and runs while the host waits for the choice.  (The
  // count array sits at the start of every variant's workspace layout.)
  StaticArgs pre;
  cc_status st = setup_args(pre, ctx, n, m, offsets, offsets_are_64bit, adj, &def, workspace, ws_bytes, labels_out,
                            num_components_dev, hip_stream);
  if (st != CC_OK) return st;
  st = select_arm(ctx, n, m, offsets, offsets_are_64bit, adj, params_dev, K, arms, norm_host, workspace, ws_bytes,
                  hip_stream, feat, &chosen, &use, &pre);
  if (st != CC_OK) return st;
  if (features_host) memcpy(features_host, feat, sizeof(feat));
  if (chosen_host) *chosen_host = chosen;
  StaticArgs a;
  st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, &use, workspace, ws_bytes, labels_out,
                  num_components_dev, hip_stream);
  if (st != CC_OK) return st;
  a.skip_init = true;
  return static_run(a);
}

}  // extern "C"
