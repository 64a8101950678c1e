// CSR validator: the preconditions every static call assumes but does not
// check on the device.
//
// The skip of the most frequent sampled component (Section 3.1, Algorithm 1)
// is only correct on a symmetric graph: a vertex outside L_max must see its
// edge to L_max from its own row, because the rows of L_max are never
// visited (appendix "Correctness for Sampling Algorithms").  The static
// kernels index the parent array with adjacency ids and the adjacency with
// offsets, so a malformed CSR faults there instead of returning an error.
// This pass checks, reading each array at most twice:
//   pass 1 (structure): offsets[0] = 0, offsets[n] = m, every row's
//     0 <= offsets[v] <= offsets[v+1] <= m, every id in [0, n), and whether
//     every row is ascending;
//   pass 2 (symmetry, only when pass 1 is clean): for every entry (v, w),
//     v occurs in row w.  With ascending rows this is a binary search in row
//     w (exact, counts the entries without a reverse); otherwise the two
//     multisets {(v, w)} and {(w, v)} are compared by a 64-bit sum of a
//     bijective hash of the ordered pair (a symmetric CSR always passes).
// Rows up to kLaneRow entries are walked by one lane, longer ones by the
// whole wave.  Entries of a malformed row are never read: a lane first
// checks that its row lies inside [0, m).
#include "cc_device.h"
#include "cc_internal.h"

namespace cc {

namespace {

constexpr int kValBlock = 256;
constexpr int kLaneRow = 32;
constexpr uint64_t kFpKey = 0x637372737966ULL;

__device__ __forceinline__ uint64_t pair_hash(int32_t a, int32_t b) {
  return sm_fin((((uint64_t)(uint32_t)a << 32) | (uint64_t)(uint32_t)b) ^ kFpKey);
}

// Position of the first entry >= x in the ascending range adj[lo, hi).
__device__ __forceinline__ int64_t lower_bound(const int32_t* adj, int64_t lo, int64_t hi, int32_t x) {
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (adj[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ void k_csr_reset(DevScalars* sc) {
  sc->csr_failed = 0;
  sc->csr_unsorted = 0;
  sc->csr_bad = 0;
  sc->csr_first = 0x7fffffffffffffffLL;
  sc->csr_fp = 0;
}

// Per-lane tallies, reduced over the wave and added once per wave.
struct Tally {
  uint32_t failed = 0;
  uint32_t unsorted = 0;
  long long bad = 0;
  long long first = 0x7fffffffffffffffLL;
  uint64_t fp = 0;
  __device__ void flag(uint32_t bit, int64_t row) {
    failed |= bit;
    first = row < first ? row : first;
  }
};

// Checks entry j of row v (value w); `next` is the following entry of the
// same row (only read by pass 1's order check, when has_next).
template <int MODE, typename I>
__device__ __forceinline__ void check_entry(Tally& t, int64_t n, const I* off, const int32_t* adj, int64_t v,
                                            int32_t w, bool has_next, int32_t next) {
  if constexpr (MODE == 0) {
    if (w < 0 || (int64_t)w >= n) {
      t.flag(CC_CSR_ID_RANGE, v);
      ++t.bad;
    }
    if (has_next && next < w) t.unsorted = 1;
  } else if constexpr (MODE == 1) {
    const int64_t lo = (int64_t)off[w], hi = (int64_t)off[w + 1];
    const int64_t p = lower_bound(adj, lo, hi, (int32_t)v);
    if (p >= hi || adj[p] != (int32_t)v) {
      t.flag(CC_CSR_ASYMMETRIC, v);
      ++t.bad;
    }
  } else {
    t.fp += pair_hash((int32_t)v, w) - pair_hash(w, (int32_t)v);
  }
}

// MODE 0: structure; 1: symmetry by binary search; 2: symmetry fingerprint.
template <int MODE, typename I>
__global__ void __launch_bounds__(kValBlock) k_csr_check(int64_t n, int64_t m, const I* __restrict__ off,
                                                         const int32_t* __restrict__ adj, DevScalars* sc) {
  const int lane = lane_id();
  Tally t;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = blockIdx.x * (int64_t)blockDim.x; base < n; base += stride) {
    const int64_t v = base + threadIdx.x;
    int64_t b = 0, e = 0;
    if (v < n) {
      b = (int64_t)off[v];
      e = (int64_t)off[v + 1];
      if constexpr (MODE == 0) {
        if (v == 0 && b != 0) t.flag(CC_CSR_OFFSET0, 0);
        if (v == n - 1 && e != m) t.flag(CC_CSR_OFFSETN, v);
        if (b < 0 || e < b || e > m) {
          t.flag(CC_CSR_MONOTONE, v);
          b = e = 0;  // never read a malformed row
        }
      }
    }
    const bool wide = (e - b) > kLaneRow;
    uint64_t bm = __ballot(wide);
    while (bm) {
      const int l = __ffsll((unsigned long long)bm) - 1;
      bm &= bm - 1;
      const int64_t rv = __shfl(v, l, kWave);
      const int64_t rb = __shfl(b, l, kWave), re = __shfl(e, l, kWave);
      for (int64_t j = rb + lane; j < re; j += kWave) {
        const bool has_next = j + 1 < re;
        check_entry<MODE, I>(t, n, off, adj, rv, adj[j], has_next, (MODE == 0 && has_next) ? adj[j + 1] : 0);
      }
    }
    if (!wide) {
      for (int64_t j = b; j < e; ++j) {
        const bool has_next = j + 1 < e;
        check_entry<MODE, I>(t, n, off, adj, v, adj[j], has_next, (MODE == 0 && has_next) ? adj[j + 1] : 0);
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    t.failed |= (uint32_t)__shfl_xor((int)t.failed, o, kWave);
    t.unsorted |= (uint32_t)__shfl_xor((int)t.unsorted, o, kWave);
    t.bad += __shfl_xor(t.bad, o, kWave);
    const long long f = __shfl_xor(t.first, o, kWave);
    t.first = f < t.first ? f : t.first;
    t.fp += (uint64_t)__shfl_xor((unsigned long long)t.fp, o, kWave);
  }
  if (lane == 0) {
    if (t.failed) {
      __hip_atomic_fetch_or(&sc->csr_failed, t.failed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t err = (t.failed & CC_CSR_ID_RANGE ? kErrBadId : 0u) |
                           (t.failed & ~(uint32_t)CC_CSR_ID_RANGE ? kErrBadCsr : 0u);
      __hip_atomic_fetch_or(&sc->error, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_min(&sc->csr_first, t.first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (t.unsorted) __hip_atomic_fetch_or(&sc->csr_unsorted, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t.bad) add64(&sc->csr_bad, t.bad);
    if (MODE == 2 && t.fp)
      __hip_atomic_fetch_add(&sc->csr_fp, (unsigned long long)t.fp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int MODE, typename I>
void launch_check(int64_t n, int64_t m, const void* off, const int32_t* adj, DevScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL((k_csr_check<MODE, I>), dim3(grid_for(n, kValBlock, 8192)), dim3(kValBlock), 0, s, n, m,
                     (const I*)off, adj, sc);
}

template <int MODE>
void launch_mode(int64_t n, int64_t m, const void* off, bool o64, const int32_t* adj, DevScalars* sc,
                 hipStream_t s) {
  if (o64) launch_check<MODE, int64_t>(n, m, off, adj, sc, s);
  else launch_check<MODE, int32_t>(n, m, off, adj, sc, s);
}

}  // namespace

}  // namespace cc

using namespace cc;

extern "C" {

cc_status cc_validate_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                          const int32_t* adj, int check_symmetric, cc_csr_report* report, void* hip_stream) {
  if (!ctx || !report) return fail(CC_EINVAL, "NULL ctx or report");
  if (n < 1 || n > 0x7fffffffLL || m < 0) return fail(CC_EINVAL, "bad n or m");
  if (!offsets || (m > 0 && !adj)) return fail(CC_EINVAL, "NULL pointer");
  if (!offsets_are_64bit && m > 0x7fffffffLL) return fail(CC_EINVAL, "m needs 64-bit offsets");
  *report = cc_csr_report{};
  report->first_bad_row = -1;
  // an error word left by an earlier call is reported, not mixed into this check
  cc_status st = cc_ctx_sync_status(ctx);
  if (st != CC_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  DevScalars* sc = ctx->dev;
  const bool o64 = offsets_are_64bit != 0;
  hipLaunchKernelGGL(k_csr_reset, dim3(1), dim3(1), 0, s, sc);
  launch_mode<0>(n, m, offsets, o64, adj, sc, s);
  CC_LAUNCH_CHECK();
  CC_HIP(hipMemcpyAsync(ctx->host, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
  CC_HIP(hipStreamSynchronize(s));
  uint32_t failed = ctx->host->csr_failed;
  int64_t bad = ctx->host->csr_bad;
  int64_t first = ctx->host->csr_first;
  report->rows_sorted = ctx->host->csr_unsorted ? 0 : 1;
  if (check_symmetric && failed == 0 && m > 0) {
    report->symmetry_checked = report->rows_sorted ? 1 : 2;
    if (report->rows_sorted) launch_mode<1>(n, m, offsets, o64, adj, sc, s);
    else launch_mode<2>(n, m, offsets, o64, adj, sc, s);
    CC_LAUNCH_CHECK();
    CC_HIP(hipMemcpyAsync(ctx->host, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
    CC_HIP(hipStreamSynchronize(s));
    failed = ctx->host->csr_failed;
    bad = ctx->host->csr_bad;
    first = ctx->host->csr_first;
    if (ctx->host->csr_fp != 0) failed |= CC_CSR_ASYMMETRIC;
  } else if (check_symmetric && failed == 0) {
    report->symmetry_checked = 1;  // no entries: trivially symmetric
  }
  report->failed = failed;
  report->bad_entries = bad;
  report->first_bad_row = failed ? (first == 0x7fffffffffffffffLL ? -1 : first) : -1;
  // the verdict is returned here, so the error word this pass set is cleared
  const uint32_t zero = 0;
  CC_HIP(hipMemcpyAsync(&sc->error, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
  CC_HIP(hipStreamSynchronize(s));
  if (failed)
    return fail(CC_EDEVICE, "malformed CSR: checks 0x%x failed (%lld bad entries, first at row %lld)", failed,
                (long long)bad, (long long)report->first_bad_row);
  return CC_OK;
}

}  // extern "C"
