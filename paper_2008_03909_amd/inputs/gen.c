/*
 * Seeded synthetic graph inputs (host C, OpenMP).
 *
 * This module only draws inputs: edge lists of the graph families the
 * connectivity workloads are built from, and streams of query pairs.  It
 * holds none of the connectivity method's arithmetic; both the device path
 * and the CPU oracle consume what it produces.
 *
 * Randomness: every draw is an output of the splitmix64 generator (Steele,
 * Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA
 * 2014) used in counter mode: output i of the generator seeded with state s
 * is fin(s + (i+1)*GAMMA), where fin is its 64-bit finalizer.  A stream key
 * is output `stream` of the generator seeded with the user seed, so every
 * draw is addressable by (seed, stream, index) and generation parallelises
 * without changing results.
 *
 * Edge lists are undirected pairs (u, v), int32, possibly with self-loops
 * and duplicates; building adjacency from them is the consumer's job.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t fin64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t draw(uint64_t state, uint64_t i) { return fin64(state + (i + 1) * GAMMA); }
static inline uint64_t stream_key(uint64_t seed, uint64_t stream) { return draw(seed, stream); }
/* uniform in [0, bound) from the top 32 bits (multiply-shift) */
static inline uint32_t hi_bounded(uint64_t r, uint32_t bound) {
  return (uint32_t)(((r >> 32) * (uint64_t)bound) >> 32);
}
static inline uint32_t lo_bounded(uint64_t r, uint32_t bound) {
  return (uint32_t)(((r & 0xffffffffULL) * (uint64_t)bound) >> 32);
}

enum { STREAM_ER = 1, STREAM_RMAT = 2, STREAM_GRID = 3, STREAM_PAIRS = 4, STREAM_SHUFFLE = 5,
       STREAM_PERM = 6 };

uint64_t gen_splitmix_draw(uint64_t seed, uint64_t stream, uint64_t i) {
  return draw(stream_key(seed, stream), i);
}

/* Erdos-Renyi multigraph: num_pairs pairs, both endpoints uniform in [0,n).
 * Endpoint u comes from the high 32 bits of one draw, v from its low 32 bits. */
void gen_er(int64_t n, int64_t num_pairs, uint64_t seed, int32_t* u, int32_t* v) {
  const uint64_t key = stream_key(seed, STREAM_ER);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < num_pairs; ++i) {
    uint64_t r = draw(key, (uint64_t)i);
    u[i] = (int32_t)hi_bounded(r, (uint32_t)n);
    v[i] = (int32_t)lo_bounded(r, (uint32_t)n);
  }
}

/* Uniform random vertex pairs (query workloads); same law as gen_er on its own stream. */
void gen_pairs(int64_t n, int64_t num_pairs, uint64_t seed, int32_t* a, int32_t* b) {
  const uint64_t key = stream_key(seed, STREAM_PAIRS);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < num_pairs; ++i) {
    uint64_t r = draw(key, (uint64_t)i);
    a[i] = (int32_t)hi_bounded(r, (uint32_t)n);
    b[i] = (int32_t)lo_bounded(r, (uint32_t)n);
  }
}

/* R-MAT (Chakrabarti, Zhan, Faloutsos 2004): n = 2^scale; each tuple descends
 * `scale` levels of the adjacency matrix and at every level picks a quadrant
 * with probabilities (a, b, c, 1-a-b-c) = (top-left, top-right, bottom-left,
 * bottom-right).  Level l of tuple i uses draw i*scale + l; the quadrant is
 * picked from the top 53 bits as a double in [0,1).  No noise, no relabelling. */
void gen_rmat(int32_t scale, int64_t num_tuples, double a, double b, double c, uint64_t seed,
              int32_t* u, int32_t* v) {
  const uint64_t key = stream_key(seed, STREAM_RMAT);
  const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < num_tuples; ++i) {
    uint32_t uu = 0, vv = 0;
    for (int32_t l = 0; l < scale; ++l) {
      uint64_t r = draw(key, (uint64_t)i * (uint64_t)scale + (uint64_t)l);
      double x = (double)(r >> 11) * (1.0 / 9007199254740992.0);
      uint32_t bit = 1u << (scale - 1 - l);
      if (x < a) {
      } else if (x < ab) {
        vv |= bit;
      } else if (x < abc) {
        uu |= bit;
      } else {
        uu |= bit;
        vv |= bit;
      }
    }
    u[i] = (int32_t)uu;
    v[i] = (int32_t)vv;
  }
}

static inline int keep_edge(uint64_t r, double p) {
  if (p >= 1.0) return 1;
  if (p <= 0.0) return 0;
  /* keep iff r < p * 2^64 */
  return (double)r < p * 18446744073709551616.0;
}

/* Bond percolation on the non-periodic L^dims lattice (dims = 2 or 3).
 * Vertex id = x + L*y (+ L*L*z).  Lattice edges are enumerated direction by
 * direction; edge e is kept iff draw e of the grid stream is < p * 2^64.
 * Returns the number of kept edges; u/v may be NULL to only count. */
int64_t gen_grid(int32_t dims, int64_t L, double p, uint64_t seed, int32_t* u, int32_t* v) {
  const uint64_t key = stream_key(seed, STREAM_GRID);
  int64_t out = 0, e = 0;
  if (dims == 2) {
    for (int d = 0; d < 2; ++d) {
      for (int64_t y = 0; y < (d == 1 ? L - 1 : L); ++y)
        for (int64_t x = 0; x < (d == 0 ? L - 1 : L); ++x, ++e) {
          if (!keep_edge(draw(key, (uint64_t)e), p)) continue;
          int64_t a = x + L * y;
          int64_t b = d == 0 ? a + 1 : a + L;
          if (u) { u[out] = (int32_t)a; v[out] = (int32_t)b; }
          ++out;
        }
    }
  } else {
    for (int d = 0; d < 3; ++d) {
      for (int64_t z = 0; z < (d == 2 ? L - 1 : L); ++z)
        for (int64_t y = 0; y < (d == 1 ? L - 1 : L); ++y)
          for (int64_t x = 0; x < (d == 0 ? L - 1 : L); ++x, ++e) {
            if (!keep_edge(draw(key, (uint64_t)e), p)) continue;
            int64_t a = x + L * (y + L * z);
            int64_t b = d == 0 ? a + 1 : (d == 1 ? a + L : a + L * L);
            if (u) { u[out] = (int32_t)a; v[out] = (int32_t)b; }
            ++out;
          }
    }
  }
  return out;
}

/* Uniform random permutation of [0, n) by Fisher-Yates driven by the
 * permutation stream: for i = n-1 .. 1 swap perm[i] with perm[j],
 * j = (draw i) mod (i+1). */
void gen_permutation(int64_t n, uint64_t seed, int32_t* perm) {
  const uint64_t key = stream_key(seed, STREAM_PERM);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)(draw(key, (uint64_t)i) % (uint64_t)(i + 1));
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
}

/* In-place Fisher-Yates shuffle of a pair list (edge streams). */
void gen_shuffle_pairs(int64_t count, uint64_t seed, int32_t* u, int32_t* v) {
  const uint64_t key = stream_key(seed, STREAM_SHUFFLE);
  for (int64_t i = count - 1; i > 0; --i) {
    int64_t j = (int64_t)(draw(key, (uint64_t)i) % (uint64_t)(i + 1));
    int32_t t = u[i]; u[i] = u[j]; u[j] = t;
    t = v[i]; v[i] = v[j]; v[j] = t;
  }
}

/* Keep each pair once: drop pairs with u == v and pairs whose (min,max) was
 * already seen earlier in the list is NOT done here (consumers handle
 * duplicates); this helper only canonicalises orientation u < v in place and
 * drops self-loops, returning the new count.  Used to turn an edge list into
 * an insertion stream where each pair is one undirected insert. */
int64_t gen_orient_drop_loops(int64_t count, int32_t* u, int32_t* v) {
  int64_t out = 0;
  for (int64_t i = 0; i < count; ++i) {
    int32_t a = u[i], b = v[i];
    if (a == b) continue;
    if (a > b) { int32_t t = a; a = b; b = t; }
    u[out] = a; v[out] = b; ++out;
  }
  return out;
}

/* Symmetric edge weights: the weight of the undirected pair {a, b} is
 * mean * (-ln U), U uniform in (0, 1) from the top 53 bits of draw
 * min(a,b) * n + max(a,b) of the weight stream -- an exponential law, the
 * same for both orientations and for every copy of the pair.  Written as
 * float (the weighted CSR's element type). */
#include <math.h>
void gen_pair_weights(int64_t n, int64_t count, const int32_t* a, const int32_t* b, double mean, uint64_t seed,
                      float* w) {
  const uint64_t key = stream_key(seed, 7);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < count; ++i) {
    const int64_t x = a[i] < b[i] ? a[i] : b[i];
    const int64_t y = a[i] < b[i] ? b[i] : a[i];
    const uint64_t r = draw(key, (uint64_t)x * (uint64_t)n + (uint64_t)y);
    const double u = ((double)(r >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    w[i] = (float)(-mean * log(u));
  }
}
