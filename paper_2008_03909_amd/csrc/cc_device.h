// Device-side building blocks for the connectivity kernels (gfx950, wave64).
//
// Parent arrays are int32 and are shared by every wave of a launch, so every
// access that the algorithms treat as racy (the starred reads and CAS of the
// union-find pseudocode in the ConnectIt appendix "Union Find Algorithms")
// is an agent-scope atomic: relaxed loads compile to `global_load ... sc1`,
// which cannot hit a stale line, and CAS / min are agent-scope RMWs.  The
// invariant that every link points to a smaller id (P[x] <= x) keeps the
// forest acyclic and makes each root its tree's minimum, which is what lets
// the final labels be the canonical minimum-id labels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cc {

constexpr int kWave = 64;

// This block's share of a sweep over [0, n) (see xcd_grid): items
// base + threadIdx.x, then steps of `step` while below `end`; `base` is the
// same for the whole block, so loops over it keep block-uniform control.
struct XcdSweep {
  int64_t base, end, step;
};
__device__ __forceinline__ XcdSweep xcd_sweep(int64_t n) {
  const int64_t G = gridDim.x, B = blockDim.x;
  if (G < 8 || G % 8) return XcdSweep{blockIdx.x * B, n, G * B};
  const int64_t x = blockIdx.x % 8, i = blockIdx.x / 8;
  const int64_t span = ((n + 7) / 8 + B - 1) / B * B;
  const int64_t lo = x * span < n ? x * span : n, hi = lo + span < n ? lo + span : n;
  return XcdSweep{lo + i * B, hi, G / 8 * B};
}

__device__ __forceinline__ int32_t ld(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool cas(int32_t* p, int32_t expected, int32_t desired) {
  return __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
}
// writeMin; returns the previous value.
__device__ __forceinline__ int32_t amin(int32_t* p, int32_t v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t aor(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long add64(long long* p, long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ldu(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- splitmix64 in counter mode (Steele, Lea, Flood, OOPSLA 2014) --------
// Output i of the generator seeded with state s is fin(s + (i+1) * gamma).
__host__ __device__ __forceinline__ uint64_t sm_fin(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
__host__ __device__ __forceinline__ uint64_t sm_out(uint64_t state, uint64_t i) {
  return sm_fin(state + (i + 1) * 0x9E3779B97F4A7C15ULL);
}
// Stream tags for the method's own random draws.
constexpr uint64_t kTagKout = 0x6b6f7574ULL;  // "kout"
constexpr uint64_t kTagBfs = 0x626673ULL;     // "bfs"
constexpr uint64_t kTagLdd = 0x6c6464ULL;     // "ldd"

// ---- find options (ConnectIt appendix, "Find Algorithms") ----------------
enum FindKind { kFindNaive = 0, kFindSplit = 1, kFindHalve = 2, kFindCompress = 3 };
enum SpliceKind { kSplitOne = 0, kHalveOne = 1, kSpliceAtomic = 2 };

// FindNaive: follow parents to the root, no writes.
__device__ __forceinline__ int32_t find_naive(int32_t* P, int32_t u) {
  int32_t p = ld(P + u);
  while (p != u) {
    u = p;
    p = ld(P + u);
  }
  return u;
}

// FindAtomicSplit: point each visited node at its grandparent, then step to
// the old parent.  FindAtomicHalve: same CAS, then step to the node's
// (possibly new) parent.  Both re-read v and w every iteration.
template <int KIND>
__device__ __forceinline__ int32_t find_split_halve(int32_t* P, int32_t u) {
  while (true) {
    int32_t v = ld(P + u);
    int32_t w = ld(P + v);
    if (v == w) return v;
    cas(P + u, v, w);
    u = (KIND == kFindSplit) ? v : ld(P + u);
  }
}

// FindCompress: find the root, then point every node of the walked path
// whose parent is still above the root directly at the root.
__device__ __forceinline__ int32_t find_compress(int32_t* P, int32_t u) {
  int32_t r = u;
  int32_t p = ld(P + r);
  if (p == r) return r;
  while (p != r) {
    r = p;
    p = ld(P + r);
  }
  int32_t j = ld(P + u);
  while (j > r) {
    st(P + u, r);
    u = j;
    j = ld(P + u);
  }
  return r;
}

template <int FIND>
__device__ __forceinline__ int32_t find(int32_t* P, int32_t u) {
  if constexpr (FIND == kFindNaive) return find_naive(P, u);
  else if constexpr (FIND == kFindCompress) return find_compress(P, u);
  else return find_split_halve<FIND>(P, u);
}

// ---- UF-Async (Jayanti-Tarjan style; appendix "UF-Async") ----------------
// Find both roots; CAS the larger root onto the smaller; retry on failure.
// Returns the root this call hooked, or -1 if u and v were already joined.
template <int FIND>
__device__ __forceinline__ int32_t union_async(int32_t* P, int32_t u, int32_t v) {
  while (true) {
    int32_t pu = find<FIND>(P, u);
    int32_t pv = find<FIND>(P, v);
    if (pu == pv) return -1;
    if (pu < pv) {
      int32_t t = pu;
      pu = pv;
      pv = t;
    }
    if (ld(P + pu) == pu && cas(P + pu, pu, pv)) return pu;
  }
}

// ---- UF-Rem-CAS (lock-free Rem; appendix "UF-Rem-CAS") --------------------
// Walk both paths upward comparing parents; the side with the larger parent
// moves.  If it is a root, CAS-hook it under the other side's parent;
// otherwise take one splice step (SplitAtomicOne, HalveAtomicOne or
// SpliceAtomic).  After a successful hook the non-naive compress options
// re-run their find on both endpoints.  Returns the root this call hooked
// (the spanning-forest slot of edge (u, v)), or -1 if it linked nothing.
// union_rem_from takes the parents of u and v already read by the caller
// (so that a caller can overlap those loads across several edges).
template <int SPLICE, int FIND>
__device__ __forceinline__ int32_t union_rem_from(int32_t* P, int32_t u, int32_t v, int32_t pu0, int32_t pv0) {
  int32_t ru = u, rv = v;
  bool first = true;
  while (true) {
    int32_t pu = first ? pu0 : ld(P + ru);
    int32_t pv = first ? pv0 : ld(P + rv);
    first = false;
    if (pu == pv) return -1;
    if (pu < pv) {
      int32_t t = ru;
      ru = rv;
      rv = t;
      t = pu;
      pu = pv;
      pv = t;
    }
    // now P[ru] = pu > pv = P[rv]
    if (pu == ru) {
      if (cas(P + ru, ru, pv)) {
        if constexpr (FIND != kFindNaive) {
          find<FIND>(P, u);
          find<FIND>(P, v);
        }
        return ru;
      }
      continue;  // lost the race: re-read both parents
    }
    if constexpr (SPLICE == kSpliceAtomic) {
      // Splice: re-parent ru under rv's parent (smaller than ru's parent).
      cas(P + ru, pu, pv);
      ru = pu;
    } else {
      // One path-split / path-halve step at ru.
      int32_t w = ld(P + pu);
      if (pu != w) cas(P + ru, pu, w);
      ru = (SPLICE == kSplitOne) ? pu : w;
    }
  }
}

// UF-Rem-CAS with FindNaive whose SplitAtomicOne step can be switched off
// per call: without it the walk only reads parents, and the only writes are
// the hooking CASes at roots (used by k-out sampling, see k_kout).
__device__ __forceinline__ int32_t union_rem_opt_split(int32_t* P, int32_t u, int32_t v, bool split) {
  int32_t ru = u, rv = v;
  while (true) {
    int32_t pu = ld(P + ru);
    int32_t pv = ld(P + rv);
    if (pu == pv) return -1;
    if (pu < pv) {
      int32_t t = ru;
      ru = rv;
      rv = t;
      t = pu;
      pu = pv;
      pv = t;
    }
    if (pu == ru) {
      if (cas(P + ru, ru, pv)) return ru;
      continue;
    }
    if (split) {
      const int32_t w = ld(P + pu);
      if (pu != w) cas(P + ru, pu, w);
    }
    ru = pu;
  }
}

template <int SPLICE, int FIND>
__device__ __forceinline__ int32_t union_rem(int32_t* P, int32_t u, int32_t v) {
  return union_rem_from<SPLICE, FIND>(P, u, v, ld(P + u), ld(P + v));
}

// ---- UF-Early (Section 3.3, the variants of UF-Async) ----------------------
// Walk both paths together: the larger of the two current nodes moves up;
// once it is a root it is hooked (CAS) under the other node, which is
// smaller and, since every tree's root is its minimum, in another tree.
// Equal nodes: already joined.  With a compress find, both endpoints are
// found again after a hook.  Returns the hooked root or -1.
template <int FIND>
__device__ __forceinline__ int32_t union_early(int32_t* P, int32_t u, int32_t v) {
  int32_t x = u, y = v;
  while (true) {
    if (x == y) return -1;
    if (x < y) {
      const int32_t t = x;
      x = y;
      y = t;
    }
    const int32_t px = ld(P + x);
    if (px == x) {
      if (cas(P + x, x, y)) {
        if constexpr (FIND != kFindNaive) {
          find<FIND>(P, u);
          find<FIND>(P, v);
        }
        return x;
      }
      continue;  // lost the race: read x's new parent
    }
    x = px;
  }
}

// ---- UF-Hooks ------------------------------------------------------------------
// As UF-Async, but the CAS that claims a root goes to an auxiliary array H
// (H[r] = -1 while r is unclaimed); the winner then writes P[r] with a plain
// store that no other thread contends for.  A root is hooked from the
// moment its claim succeeds, so finds follow H[r] from a claimed root
// whose P[r] is not written yet: no thread ever waits for another's store
// (a lane spinning on a store that its own wave's exiting lane has yet to
// issue would never see it).
template <int FIND>
__device__ __forceinline__ int32_t find_hooks(int32_t* P, const int32_t* H, int32_t u) {
  while (true) {
    const int32_t r = find<FIND>(P, u);
    const int32_t h = ld(H + r);
    if (h < 0) return r;
    u = h;
  }
}

template <int FIND>
__device__ __forceinline__ int32_t union_hooks(int32_t* P, int32_t* H, int32_t u, int32_t v) {
  while (true) {
    int32_t pu = find_hooks<FIND>(P, H, u);
    int32_t pv = find_hooks<FIND>(P, H, v);
    if (pu == pv) return -1;
    if (pu < pv) {
      const int32_t t = pu;
      pu = pv;
      pv = t;
    }
    if (cas(H + pu, -1, pv)) {
      st(P + pu, pv);
      return pu;
    }
  }
}

// Union dispatch.  ALG 0 = Rem-CAS (SPLICE, FIND), 1 = Async (FIND),
// 2 = Early (FIND), 3 = Hooks (FIND; H is its claim array, else unused).
// Returns the hooked root or -1.
template <int ALG, int SPLICE, int FIND>
__device__ __forceinline__ int32_t unite(int32_t* P, int32_t u, int32_t v, int32_t* H = nullptr) {
  if constexpr (ALG == 0) return union_rem<SPLICE, FIND>(P, u, v);
  else if constexpr (ALG == 1) return union_async<FIND>(P, u, v);
  else if constexpr (ALG == 2) return union_early<FIND>(P, u, v);
  else return union_hooks<FIND>(P, H, u, v);
}

// Spanning forest: the edge that hooked root r is stored at slot r (each
// root is hooked at most once, so no slot is written twice).
__device__ __forceinline__ void forest_record(int2* hook, int32_t r, int32_t u, int32_t v) {
  if (hook && r >= 0) hook[r] = make_int2(u, v);
}

// ---- wave helpers -----------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

}  // namespace cc
