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
// Features (16 FP32, host-computed from device reductions):
//   0 log2 n          1 log2(m+1)         2 m/n               3 degree CV
//   4 max/mean deg    5 frac deg 0        6 frac deg 1        7 frac deg <= 2
//   8 degree skew     9 k-out L_max frac  10 k-out comps / n  11 k-out inter-component edge frac (16384 sampled edges)
//   12 BFS levels (<= 8) from a seeded source   13 BFS coverage at the cap
//   14 [m/n < 3]      15 log2(max deg + 1)
// The k-out sample (k = 2 hybrid, the default variant's) is left in the
// caller's label buffer, so an arm with that sampler continues from it.
//
// MLP: parameters packed as BF16 [W1 16x64 | b1 64 | W2 64x64 | b2 64 |
// W3 64xK | b3 K] (row-major, input index first).  Inputs and hidden
// activations are rounded to BF16; every product is accumulated in FP32;
// outputs are FP32 predicted log-time ratios; ReLU between layers.  The
// backward pass treats the BF16 rounding as identity (straight-through) and
// the ReLU derivative at 0 as 0.
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

// One block per row.  cache (nullable): per row [z1 64 | a1 64 | z2 64 | a2 64].
__global__ void __launch_bounds__(kH) k_mlp_forward(const uint16_t* __restrict__ params, int K, int B,
                                                    const float* __restrict__ X, float* __restrict__ Y,
                                                    float* __restrict__ cache) {
  __shared__ float x[kIn], a1[kH], a2[kH];
  const int r = blockIdx.x, t = threadIdx.x;
  if (r >= B) return;
  const MlpView P = mlp_view(params, K);
  if (t < kIn) x[t] = bf16_round(X[(int64_t)r * kIn + t]);
  __syncthreads();
  float z = bf16_to_f32(P.b1[t]);
  for (int i = 0; i < kIn; ++i) z += x[i] * bf16_to_f32(P.W1[i * kH + t]);
  const float h1 = bf16_round(z > 0.f ? z : 0.f);
  a1[t] = h1;
  if (cache) {
    cache[(int64_t)r * 4 * kH + t] = z;
    cache[(int64_t)r * 4 * kH + kH + t] = h1;
  }
  __syncthreads();
  z = bf16_to_f32(P.b2[t]);
  for (int i = 0; i < kH; ++i) z += a1[i] * bf16_to_f32(P.W2[i * kH + t]);
  const float h2 = bf16_round(z > 0.f ? z : 0.f);
  a2[t] = h2;
  if (cache) {
    cache[(int64_t)r * 4 * kH + 2 * kH + t] = z;
    cache[(int64_t)r * 4 * kH + 3 * kH + t] = h2;
  }
  __syncthreads();
  for (int j = t; j < K; j += kH) {
    float y = bf16_to_f32(P.b3[j]);
    for (int i = 0; i < kH; ++i) y += a2[i] * bf16_to_f32(P.W3[i * K + j]);
    Y[(int64_t)r * K + j] = y;
  }
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

// Per-block partials: [sum d, sum d^2, sum d^3, max d, #d==0, #d==1, #d<=2, 0].
template <typename I>
__global__ void __launch_bounds__(256) k_deg_stats(int64_t n, const I* __restrict__ off, double* __restrict__ part) {
  __shared__ double red[8][256 / kWave];
  double s1 = 0, s2 = 0, s3 = 0, mx = 0, c0 = 0, c1 = 0, c2 = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n; v += stride) {
    const double d = (double)((int64_t)off[v + 1] - (int64_t)off[v]);
    s1 += d;
    s2 += d * d;
    s3 += d * d * d;
    mx = d > mx ? d : mx;
    c0 += d == 0.0;
    c1 += d == 1.0;
    c2 += d <= 2.0;
  }
  double vals[7] = {s1, s2, s3, mx, c0, c1, c2};
  for (int q = 0; q < 7; ++q) {
    double x = vals[q];
    for (int o = 32; o > 0; o >>= 1) {
      const double y = __shfl_xor(x, o, kWave);
      x = (q == 3) ? (y > x ? y : x) : x + y;
    }
    if (lane_id() == 0) red[q][threadIdx.x / kWave] = x;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int q = threadIdx.x;
    double x = red[q][0];
    for (int w = 1; w < 256 / kWave; ++w) x = (q == 3) ? (red[q][w] > x ? red[q][w] : x) : x + red[q][w];
    part[(int64_t)blockIdx.x * 8 + q] = x;
  }
}

// Sampled-labelling statistics: [#roots, #label == lmax, #sampled edges with
// different endpoint labels, #sampled edges].
template <typename I>
__global__ void __launch_bounds__(256) k_label_stats(int64_t n, int64_t m, const I* __restrict__ off,
                                                     const int32_t* __restrict__ adj,
                                                     const int32_t* __restrict__ P, const DevScalars* sc,
                                                     uint64_t key, int nsamples,
                                                     unsigned long long* __restrict__ out) {
  const int32_t L = sc->lmax;
  unsigned long long roots = 0, inl = 0, diff = 0, samp = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  for (int64_t v = gid; v < n; v += stride) {
    const int32_t p = P[v];
    roots += p == (int32_t)v;
    inl += p == L;
  }
  if (m > 0)
    for (int64_t i = gid; i < nsamples; i += stride) {
      const int64_t e = (int64_t)(sm_out(key, (uint64_t)i) % (uint64_t)m);
      int64_t lo = 0, hi = n - 1;  // owner: largest v with off[v] <= e
      while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if ((int64_t)off[mid] <= e) lo = mid;
        else hi = mid - 1;
      }
      diff += P[lo] != P[adj[e]];
      ++samp;
    }
  roots = wave_sum(roots);
  inl = wave_sum(inl);
  diff = wave_sum(diff);
  samp = wave_sum(samp);
  if (lane_id() == 0) {
    if (roots) atomicAdd(out + 0, roots);
    if (inl) atomicAdd(out + 1, inl);
    if (diff) atomicAdd(out + 2, diff);
    if (samp) atomicAdd(out + 3, samp);
  }
}

__global__ void k_zero_u64(unsigned long long* p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0ull;
}

constexpr int kFeatBlocks = 512;
constexpr int kIcSamples = 16384;
constexpr int kBfsFeatureCap = 8;
constexpr uint64_t kTagFeat = 0x66656174ULL;  // "feat"

template <typename I>
static cc_status features_impl(StaticArgs& a, float* feat) {
  // degree moments: kFeatBlocks * 8 doubles at the start of the selector area
  double* part = (double*)(a.ws + a.L.mlp);
  hipLaunchKernelGGL(k_deg_stats<I>, dim3(kFeatBlocks), dim3(256), 0, a.s, a.n, (const I*)a.off, part);
  CC_LAUNCH_CHECK();
  std::vector<double> hp(kFeatBlocks * 8);
  CC_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * 8, hipMemcpyDeviceToHost, a.s));
  // k-out sample into the caller's label buffer
  cc_status st = static_sample_only(a);
  if (st != CC_OK) return st;
  unsigned long long* ls = (unsigned long long*)(a.ws + a.L.mlp + kFeatBlocks * 8 * sizeof(double));
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, a.s, ls, 4);
  hipLaunchKernelGGL(k_label_stats<I>, dim3(kFeatBlocks), dim3(256), 0, a.s, a.n, a.m, (const I*)a.off, a.adj,
                     (const int32_t*)a.P, (const DevScalars*)a.ctx->dev, sm_out(a.v->seed, kTagFeat), kIcSamples,
                     ls);
  CC_LAUNCH_CHECK();
  unsigned long long lsh[4];
  CC_HIP(hipMemcpyAsync(lsh, ls, sizeof(lsh), hipMemcpyDeviceToHost, a.s));
  CC_HIP(hipStreamSynchronize(a.s));
  // capped BFS from a seeded source (the labels in P are left untouched)
  int64_t reached = 0;
  int32_t levels = 0;
  const int32_t src = (int32_t)(sm_out(sm_out(a.v->seed, kTagFeat), 1) % (uint64_t)a.n);
  st = bfs_probe<I>(a, src, kBfsFeatureCap, &reached, &levels);
  if (st != CC_OK) return st;
  double s1 = 0, s2 = 0, s3 = 0, mx = 0, c0 = 0, c1 = 0, c2 = 0;
  for (int b = 0; b < kFeatBlocks; ++b) {
    const double* p = &hp[b * 8];
    s1 += p[0], s2 += p[1], s3 += p[2], mx = p[3] > mx ? p[3] : mx, c0 += p[4], c1 += p[5], c2 += p[6];
  }
  const double n = (double)a.n, m = (double)a.m;
  const double mean = s1 / n;
  const double var = s2 / n - mean * mean > 0 ? s2 / n - mean * mean : 0.0;
  const double sd = std::sqrt(var);
  const double skew = sd > 0 ? (s3 / n - 3 * mean * var - mean * mean * mean) / (sd * sd * sd) : 0.0;
  const double lmax_size = (double)a.ctx->host->lmax_size;
  feat[0] = (float)std::log2(n);
  feat[1] = (float)std::log2(m + 1.0);
  feat[2] = (float)(m / n);
  feat[3] = (float)(mean > 0 ? sd / mean : 0.0);
  feat[4] = (float)(mean > 0 ? mx / mean : 0.0);
  feat[5] = (float)(c0 / n);
  feat[6] = (float)(c1 / n);
  feat[7] = (float)(c2 / n);
  feat[8] = (float)(skew > 1e6 ? 1e6 : skew);
  feat[9] = (float)(lmax_size / n);
  feat[10] = (float)((double)lsh[0] / n);
  feat[11] = (float)(lsh[3] ? (double)lsh[2] / (double)lsh[3] : 0.0);
  feat[12] = (float)levels;
  feat[13] = (float)((double)reached / n);
  feat[14] = (float)(m / n < 3.0 ? 1.0 : 0.0);
  feat[15] = (float)std::log2(mx + 1.0);
  return CC_OK;
}

static cc_status features(StaticArgs& a, float* feat) {
  // The sample step resolves lmax into ctx->dev; read it for feature 9.
  cc_status st = a.o64 ? features_impl<int64_t>(a, feat) : features_impl<int32_t>(a, feat);
  return st;
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
                            const int32_t* adj, void* workspace, size_t ws_bytes, int32_t* labels_scratch,
                            float* features_host, void* hip_stream) {
  if (!features_host) return fail(CC_EINVAL, "features_host is NULL");
  cc_variant v;
  cc_default_variant(&v);
  StaticArgs a;
  cc_status st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, &v, workspace, ws_bytes, labels_scratch,
                            nullptr, hip_stream);
  if (st != CC_OK) return st;
  st = features(a, features_host);
  return st;
}

cc_status cc_connectivity_auto(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                               const int32_t* adj, const uint16_t* params_dev, int32_t K, const cc_variant* arms,
                               const float* norm_host, void* workspace, size_t ws_bytes, int32_t* labels_out,
                               int64_t* num_components_dev, int32_t* chosen_host, float* features_host,
                               void* hip_stream) {
  if (params_dev && (K < 1 || K > kMaxArms || !arms || !norm_host)) return fail(CC_EINVAL, "bad selector arguments");
  cc_variant def;
  cc_default_variant(&def);
  if (params_dev)
    for (int j = 0; j < K; ++j) {
      cc_status s2 = check_variant(&arms[j], false);
      if (s2 != CC_OK) return s2;
    }
  // workspace must serve every arm
  size_t need = ws_layout(n, m, &def).total;
  if (params_dev)
    for (int j = 0; j < K; ++j) need = std::max(need, ws_layout(n, m, &arms[j]).total);
  if (!workspace || ws_bytes < need) return fail(CC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required",
                                                 ws_bytes, need);
  StaticArgs a;
  cc_status st = setup_args(a, ctx, n, m, offsets, offsets_are_64bit, adj, &def, workspace, ws_bytes, labels_out,
                            num_components_dev, hip_stream);
  if (st != CC_OK) return st;
  float feat[kIn];
  st = features(a, feat);
  if (st != CC_OK) return st;
  if (features_host) memcpy(features_host, feat, sizeof(feat));
  int chosen = -1;
  const cc_variant* use = &def;
  if (params_dev) {
    float x[kIn];
    for (int i = 0; i < kIn; ++i) x[i] = (feat[i] - norm_host[i]) / (norm_host[kIn + i] > 0 ? norm_host[kIn + i] : 1.f);
    float* dx = (float*)(a.ws + a.L.mlp + kFeatBlocks * 8 * sizeof(double) + 256);
    float* dy = dx + 64;  // K <= 128 scores
    CC_HIP(hipMemcpyAsync(dx, x, sizeof(x), hipMemcpyHostToDevice, a.s));
    hipLaunchKernelGGL(k_mlp_forward, dim3(1), dim3(kH), 0, a.s, params_dev, K, 1, (const float*)dx, dy,
                       (float*)nullptr);
    CC_LAUNCH_CHECK();
    std::vector<float> y(K);
    CC_HIP(hipMemcpyAsync(y.data(), dy, K * sizeof(float), hipMemcpyDeviceToHost, a.s));
    CC_HIP(hipStreamSynchronize(a.s));
    chosen = 0;
    for (int j = 1; j < K; ++j)
      if (y[j] < y[chosen]) chosen = j;
    use = &arms[chosen];
  }
  if (chosen_host) *chosen_host = chosen;
  // An arm with the features' own sampler continues from that sample.
  const bool same_sample = use->sample == CC_SAMPLE_KOUT && use->kout_k == def.kout_k &&
                           use->kout_mode == def.kout_mode && use->seed == def.seed;
  if (same_sample) {
    a.v = use;
    st = static_from_sample(a);
    return st;
  }
  return cc_connectivity_csr(ctx, n, m, offsets, offsets_are_64bit, adj, use, workspace, ws_bytes, labels_out,
                             num_components_dev, hip_stream);
}

}  // extern "C"
