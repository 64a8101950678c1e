/*
 * CPU oracle for graph connectivity -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, obviously-correct C.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load this library; the
 * product path never does.  It shares no code with the device library.
 *
 * What it computes (ConnectIt, Dhulipala/Hong/Shun, arXiv 2008.03909):
 *  - the connectivity labelling of Section 2 ("Graph Connectivity and
 *    Related Problems"): labels equal iff connected.  The canonical form
 *    used throughout is label[v] = the minimum vertex id reachable from v;
 *  - two independent ways to reach it (BFS sweep; sequential union-find)
 *    and a Warshall transitive closure for tiny graphs;
 *  - adjacency (CSR) construction from an undirected pair list, as the
 *    CSR format of Section 2 ("Graph Notation and Formats") describes it;
 *  - the batch-incremental semantics of Section 3.4 / Appendix
 *    "ConnectIt: Streaming": a query answered after batches B_1..B_t sees
 *    the graph E_0 + B_1 + ... + B_t;
 *  - the exact partitions produced by the two deterministic samplers
 *    (k-out with the first edge plus k-1 seeded picks, Section 3.2 and the
 *    k-out sampling algorithm of Appendix "Sampling Schemes"; BFS sampling
 *    with up to c seeded sources and the 10% success rule), each reduced to
 *    its definition: the connected components of the sampled sub-graph.
 */
#include <stdint.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---- splitmix64 in counter mode (Steele, Lea, Flood, OOPSLA 2014) -------
 * Output i of the generator seeded with state s is fin(s + (i+1)*gamma).
 * The method's random draws (k-out picks, BFS sources) are defined on this
 * generator, so the oracle implements it from that definition. */
static uint64_t sm_fin(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static uint64_t sm_out(uint64_t state, uint64_t i) { return sm_fin(state + (i + 1) * 0x9E3779B97F4A7C15ULL); }

/* ---- CSR construction ------------------------------------------------------
 * Directed edge list = both orientations of every pair with u != v; rows
 * sorted ascending; with dedup, repeated (u,v) keep one copy.  Returns m. */
static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

int64_t oracle_csr_build(int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v, int dedup,
                         int64_t* offsets, int32_t* adj) {
  int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t i = 0; i < num_pairs; ++i) {
    if (u[i] == v[i]) continue;
    deg[u[i]]++;
    deg[v[i]]++;
  }
  offsets[0] = 0;
  for (int64_t x = 0; x < n; ++x) offsets[x + 1] = offsets[x] + deg[x];
  int64_t* fill = deg; /* reuse as write cursor */
  for (int64_t x = 0; x < n; ++x) fill[x] = offsets[x];
  for (int64_t i = 0; i < num_pairs; ++i) {
    if (u[i] == v[i]) continue;
    adj[fill[u[i]]++] = v[i];
    adj[fill[v[i]]++] = u[i];
  }
  for (int64_t x = 0; x < n; ++x)
    qsort(adj + offsets[x], (size_t)(offsets[x + 1] - offsets[x]), sizeof(int32_t), cmp_i32);
  if (dedup) {
    int64_t w = 0;
    for (int64_t x = 0; x < n; ++x) {
      int64_t b = offsets[x], e = offsets[x + 1];
      offsets[x] = w;
      for (int64_t j = b; j < e; ++j)
        if (j == b || adj[j] != adj[j - 1]) adj[w++] = adj[j];
    }
    offsets[n] = w;
  }
  free(deg);
  return offsets[n];
}

/* ---- 1. BFS sweep ----------------------------------------------------------
 * Start a BFS at v = 0, 1, ..., n-1 whenever v is still unlabelled; every
 * vertex it reaches gets label v.  The first vertex of a component met by the
 * sweep is its minimum, so the labels are canonical by construction.
 * Returns the number of components. */
int64_t oracle_bfs_cc(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t* label) {
  int32_t* queue = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  for (int64_t x = 0; x < n; ++x) label[x] = -1;
  int64_t comps = 0;
  for (int64_t s = 0; s < n; ++s) {
    if (label[s] >= 0) continue;
    ++comps;
    int64_t head = 0, tail = 0;
    label[s] = (int32_t)s;
    queue[tail++] = (int32_t)s;
    while (head < tail) {
      int32_t x = queue[head++];
      for (int64_t j = offsets[x]; j < offsets[x + 1]; ++j) {
        int32_t y = adj[j];
        if (label[y] < 0) {
          label[y] = (int32_t)s;
          queue[tail++] = y;
        }
      }
    }
  }
  free(queue);
  return comps;
}

/* ---- 2. sequential union-find ------------------------------------------
 * Link the larger root under the smaller one; path halving in find.  Since
 * every link points to a smaller id, each root is its tree's minimum. */
static int32_t uf_find(int32_t* P, int32_t x) {
  while (P[x] != x) {
    P[x] = P[P[x]];
    x = P[x];
  }
  return x;
}
static void uf_union(int32_t* P, int32_t a, int32_t b) {
  int32_t ra = uf_find(P, a), rb = uf_find(P, b);
  if (ra == rb) return;
  if (ra < rb) P[rb] = ra;
  else P[ra] = rb;
}

void oracle_uf_init(int64_t n, int32_t* P) {
  for (int64_t x = 0; x < n; ++x) P[x] = (int32_t)x;
}
void oracle_uf_insert(int64_t n, int32_t* P, int64_t k, const int32_t* u, const int32_t* v) {
  (void)n;
  for (int64_t i = 0; i < k; ++i) uf_union(P, u[i], v[i]);
}
void oracle_uf_query(int64_t n, int32_t* P, int64_t q, const int32_t* a, const int32_t* b, uint8_t* out) {
  (void)n;
  for (int64_t i = 0; i < q; ++i) out[i] = (uint8_t)(uf_find(P, a[i]) == uf_find(P, b[i]));
}
int64_t oracle_uf_labels(int64_t n, int32_t* P, int32_t* label) {
  int64_t comps = 0;
  for (int64_t x = 0; x < n; ++x) {
    label[x] = uf_find(P, (int32_t)x);
    comps += label[x] == x;
  }
  return comps;
}

int64_t oracle_uf_cc(int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v, int32_t* label) {
  int32_t* P = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  oracle_uf_init(n, P);
  oracle_uf_insert(n, P, num_pairs, u, v);
  int64_t comps = oracle_uf_labels(n, P, label);
  free(P);
  return comps;
}

/* ---- 3. Warshall transitive closure, n <= 64 ---------------------------
 * R[i] = bitmask of vertices reachable from i (reflexive); label = lowest
 * set bit.  Returns -1 if n > 64. */
int64_t oracle_closure_cc(int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v, int32_t* label) {
  if (n > 64) return -1;
  uint64_t R[64];
  for (int64_t i = 0; i < n; ++i) R[i] = 1ULL << i;
  for (int64_t e = 0; e < num_pairs; ++e) {
    R[u[e]] |= 1ULL << v[e];
    R[v[e]] |= 1ULL << u[e];
  }
  for (int64_t k = 0; k < n; ++k)
    for (int64_t i = 0; i < n; ++i)
      if (R[i] >> k & 1ULL) R[i] |= R[k];
  int64_t comps = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t lo = 0;
    while (!(R[i] >> lo & 1ULL)) ++lo;
    label[i] = lo;
    comps += lo == i;
  }
  return comps;
}

/* ---- k-out sample partition --------------------------------------------
 * The sampled sub-graph keeps, for every vertex v with deg(v) > 0, the edge
 * to its first neighbour A[I[v]] and k-1 more edges A[I[v] + (r_j mod deg)],
 * r_j = output (v*k + j) of splitmix64 seeded with key, j = 1..k-1,
 * key = output 0x6b6f7574 of splitmix64 seeded with `seed`.  The sample's
 * labelling is the connected components of that sub-graph (canonical min). */
/* k-out edge choices (Section 3.2; appendix "Sampling Schemes"): mode 0
 * hybrid (the first edge, then k-1 picks), 1 afforest (the first k edges),
 * 2 pure (k picks), 3 maxdeg (the neighbour of largest degree, the first
 * such in row order, then k-1 picks).  Pick j of x is entry
 * draw(key, x*k + j) mod deg of x's row. */
int64_t oracle_kout_sample_mode(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t k, int32_t mode,
                                uint64_t seed, int32_t* label) {
  int32_t* P = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  oracle_uf_init(n, P);
  const uint64_t key = sm_out(seed, 0x6b6f7574ULL);
  for (int64_t x = 0; x < n; ++x) {
    const int64_t b = offsets[x];
    const int64_t deg = offsets[x + 1] - b;
    if (deg == 0) continue;
    for (int32_t j = 0; j < k; ++j) {
      int64_t idx;
      if (mode == 1) {
        if (j >= deg) break;
        idx = j;
      } else if (mode == 0 && j == 0) {
        idx = 0;
      } else if (mode == 3 && j == 0) {
        idx = 0;
        for (int64_t t = 1; t < deg; ++t) {
          const int32_t y = adj[b + t], z = adj[b + idx];
          if (offsets[y + 1] - offsets[y] > offsets[z + 1] - offsets[z]) idx = t;
        }
      } else {
        idx = (int64_t)(sm_out(key, (uint64_t)x * (uint64_t)k + (uint64_t)j) % (uint64_t)deg);
      }
      uf_union(P, (int32_t)x, adj[b + idx]);
    }
  }
  int64_t comps = oracle_uf_labels(n, P, label);
  free(P);
  return comps;
}

int64_t oracle_kout_sample(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t k, uint64_t seed,
                           int32_t* label) {
  return oracle_kout_sample_mode(n, offsets, adj, k, 0, seed, label);
}

/* ---- BFS sample partition ----------------------------------------------
 * Try t = 0..tries-1: source s_t = output t of splitmix64 seeded with
 * key = output 0x626673 of splitmix64 seeded with `seed`, reduced mod n.
 * The BFS reaches exactly the component of s_t; if it holds more than n/10
 * vertices (strictly: 10*size > n, in integers), the sample labels that component with its minimum
 * member and every other vertex with itself, and the source index is
 * returned.  If no try succeeds the labelling is the identity and -1 is
 * returned. */
int64_t oracle_bfs_sample(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t tries, uint64_t seed,
                          int32_t* label) {
  const uint64_t key = sm_out(seed, 0x626673ULL);
  int32_t* queue = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  uint8_t* seen = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  int64_t result = -1;
  for (int64_t x = 0; x < n; ++x) label[x] = (int32_t)x;
  for (int32_t t = 0; t < tries && n > 0; ++t) {
    int32_t s = (int32_t)(sm_out(key, (uint64_t)t) % (uint64_t)n);
    memset(seen, 0, (size_t)n);
    int64_t head = 0, tail = 0;
    int32_t mn = s;
    seen[s] = 1;
    queue[tail++] = s;
    while (head < tail) {
      int32_t x = queue[head++];
      if (x < mn) mn = x;
      for (int64_t j = offsets[x]; j < offsets[x + 1]; ++j)
        if (!seen[adj[j]]) {
          seen[adj[j]] = 1;
          queue[tail++] = adj[j];
        }
    }
    if (10 * tail > n) {
      for (int64_t i = 0; i < tail; ++i) label[queue[i]] = mn;
      result = t;
      break;
    }
  }
  free(queue);
  free(seen);
  return result;
}

/* splitmix64 output i of the generator seeded with `state` (exported so the
 * tests can derive the same seeded choices as the device does). */
uint64_t oracle_splitmix_out(uint64_t state, uint64_t i) { return sm_out(state, i); }

/* BFS from `source` for at most `cap` levels (cap <= 0: no limit); returns
 * the number of vertices reached and writes the number of levels expanded
 * (a level counts if its frontier was non-empty when expanded). */
int64_t oracle_bfs_levels(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t source, int32_t cap,
                          int32_t* levels_out) {
  int32_t* dist = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t* queue = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  for (int64_t x = 0; x < n; ++x) dist[x] = -1;
  int64_t head = 0, tail = 0;
  dist[source] = 0;
  queue[tail++] = source;
  int32_t levels = 0;
  while (head < tail) {
    int32_t x = queue[head];
    if (cap > 0 && dist[x] >= cap) break;
    if (dist[x] + 1 > levels) levels = dist[x] + 1;
    ++head;
    for (int64_t j = offsets[x]; j < offsets[x + 1]; ++j)
      if (dist[adj[j]] < 0) {
        dist[adj[j]] = dist[x] + 1;
        queue[tail++] = adj[j];
      }
  }
  free(dist);
  free(queue);
  *levels_out = levels;
  return tail;
}

/* Breadth-first search from `source` that expands whole levels only: before
 * a level is expanded, the degrees of its frontier are summed, and the
 * search stops if expanding it would take the number of scanned adjacency
 * entries above edge_budget, or when `cap` levels have been expanded or the
 * frontier is empty.  Returns the number of vertices discovered by the
 * expanded levels (the source included) and writes that number of levels.
 * Which vertices a level discovers does not depend on the scan order, so
 * both results are unique. */
int64_t oracle_bfs_budget(int64_t n, const int64_t* offsets, const int32_t* adj, int32_t source, int32_t cap,
                          int64_t edge_budget, int32_t* levels_out) {
  uint8_t* seen = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);
  int32_t* cur = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t* nxt = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int64_t nc = 1, reached = 1, scanned = 0;
  int32_t levels = 0;
  cur[0] = source;
  seen[source] = 1;
  while (nc > 0 && levels < cap) {
    int64_t fe = 0;
    for (int64_t i = 0; i < nc; ++i) fe += offsets[cur[i] + 1] - offsets[cur[i]];
    if (scanned + fe > edge_budget) break;
    int64_t nn = 0;
    for (int64_t i = 0; i < nc; ++i)
      for (int64_t j = offsets[cur[i]]; j < offsets[cur[i] + 1]; ++j)
        if (!seen[adj[j]]) {
          seen[adj[j]] = 1;
          nxt[nn++] = adj[j];
        }
    scanned += fe;
    ++levels;
    reached += nn;
    int32_t* t = cur;
    cur = nxt;
    nxt = t;
    nc = nn;
  }
  free(seen);
  free(cur);
  free(nxt);
  *levels_out = levels;
  return reached;
}

/* ---- spanning forest check (Section 2's definition of a spanning forest) --
 * A set F of k edges is a spanning forest of G iff every edge of F is an
 * edge of G, no edge of F closes a cycle (a sequential union-find over F
 * links two different trees at every edge), and F connects exactly what G
 * connects (the labels of the union-find over F equal label_g, G's
 * canonical labels).  Membership is a binary search in the row of u of the
 * CSR (rows sorted ascending).  Returns 0 if F is a spanning forest, else a
 * code naming the first failed condition: 1 an id out of range, 2 an edge
 * not in G, 3 a cycle, 4 different connectivity. */
int64_t oracle_forest_check(int64_t n, const int64_t* offsets, const int32_t* adj, const int32_t* label_g, int64_t k,
                            const int32_t* fu, const int32_t* fv) {
  int64_t code = 0;
  int32_t* P = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  int32_t* lab = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  oracle_uf_init(n, P);
  for (int64_t i = 0; i < k && !code; ++i) {
    const int32_t a = fu[i], b = fv[i];
    if (a < 0 || b < 0 || a >= n || b >= n) {
      code = 1;
      break;
    }
    int64_t lo = offsets[a], hi = offsets[a + 1];
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (adj[mid] < b) lo = mid + 1;
      else hi = mid;
    }
    if (lo >= offsets[a + 1] || adj[lo] != b) {
      code = 2;
      break;
    }
    const int32_t ra = uf_find(P, a), rb = uf_find(P, b);
    if (ra == rb) {
      code = 3;
      break;
    }
    if (ra < rb) P[rb] = ra;
    else P[ra] = rb;
  }
  if (!code) {
    oracle_uf_labels(n, P, lab);
    for (int64_t x = 0; x < n; ++x)
      if (lab[x] != label_g[x]) {
        code = 4;
        break;
      }
  }
  free(P);
  free(lab);
  return code;
}

/* ---- minimum spanning forest weight (Kruskal) ---------------------------
 * Exact MSF weight of an undirected weighted pair list: pairs sorted by
 * weight (ties by index), each pair kept iff it joins two different trees
 * of a sequential union-find.  Self-loops never join anything. */
static const double* g_msf_w;
static int cmp_by_weight(const void* a, const void* b) {
  const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  const double wx = g_msf_w[x], wy = g_msf_w[y];
  if (wx < wy) return -1;
  if (wx > wy) return 1;
  return x < y ? -1 : (x > y);
}
double oracle_msf_weight(int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v, const double* w,
                         int64_t* num_edges) {
  int64_t* idx = (int64_t*)malloc((size_t)(num_pairs > 0 ? num_pairs : 1) * sizeof(int64_t));
  int32_t* P = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  for (int64_t i = 0; i < num_pairs; ++i) idx[i] = i;
  g_msf_w = w;
  qsort(idx, (size_t)num_pairs, sizeof(int64_t), cmp_by_weight);
  oracle_uf_init(n, P);
  double total = 0.0;
  int64_t k = 0;
  for (int64_t t = 0; t < num_pairs; ++t) {
    const int64_t i = idx[t];
    const int32_t ra = uf_find(P, u[i]), rb = uf_find(P, v[i]);
    if (ra == rb) continue;
    if (ra < rb) P[rb] = ra;
    else P[ra] = rb;
    total += w[i];
    ++k;
  }
  free(idx);
  free(P);
  if (num_edges) *num_edges = k;
  return total;
}

/* Approximate MSF buckets (Section 5.1).  The bucket boundaries are
 * t_0 = W_min and t_{i+1} = t_i * (1 + eps), each product taken in double
 * and rounded down to float, so that no bucket [t_i, t_{i+1}) spans more
 * than a factor 1 + eps; an edge of weight w is in the largest i with
 * t_i <= w.  Taking the buckets in increasing order and adding a spanning
 * forest of each bucket over the components of the earlier ones is Kruskal's
 * algorithm on the weights rounded down to their bucket's boundary, so the
 * number of forest edges that fall in each bucket is the same for every
 * such forest: those counts are returned.  Returns the number of buckets
 * (at most max_buckets; -1 if more would be needed, -2 for a weight that is
 * not finite and > 0); thresholds gets nb + 1 boundaries. */
static float round_down_float(double x) {
  float f = (float)x;
  if ((double)f > x) f = nextafterf(f, -INFINITY);
  return f;
}
static const int32_t* g_bucket_of;
static int cmp_by_bucket(const void* a, const void* b) {
  const int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  const int32_t bx = g_bucket_of[x], by = g_bucket_of[y];
  if (bx != by) return bx < by ? -1 : 1;
  return x < y ? -1 : (x > y);
}
int32_t oracle_amsf_buckets(int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v, const float* w,
                            double eps, int32_t max_buckets, float* thresholds, int64_t* counts) {
  if (num_pairs == 0) return 0;
  float wmin = INFINITY, wmax = 0.0f;
  for (int64_t i = 0; i < num_pairs; ++i) {
    if (!(w[i] > 0.0f) || isinf(w[i])) return -2;
    if (w[i] < wmin) wmin = w[i];
    if (w[i] > wmax) wmax = w[i];
  }
  int32_t nb = 0;
  thresholds[0] = wmin;
  while (thresholds[nb] <= wmax) {
    if (nb == max_buckets) return -1;
    thresholds[nb + 1] = round_down_float((double)thresholds[nb] * (1.0 + eps));
    ++nb;
  }
  int32_t* bucket = (int32_t*)malloc((size_t)num_pairs * sizeof(int32_t));
  for (int64_t i = 0; i < num_pairs; ++i) {
    int32_t lo = 0, hi = nb - 1; /* largest b with thresholds[b] <= w */
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) / 2;
      if (thresholds[mid] <= w[i]) lo = mid;
      else hi = mid - 1;
    }
    bucket[i] = lo;
  }
  int64_t* idx = (int64_t*)malloc((size_t)num_pairs * sizeof(int64_t));
  int32_t* P = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
  for (int64_t i = 0; i < num_pairs; ++i) idx[i] = i;
  g_bucket_of = bucket;
  qsort(idx, (size_t)num_pairs, sizeof(int64_t), cmp_by_bucket);
  oracle_uf_init(n, P);
  for (int32_t b = 0; b < nb; ++b) counts[b] = 0;
  for (int64_t t = 0; t < num_pairs; ++t) {
    const int64_t i = idx[t];
    const int32_t ra = uf_find(P, u[i]), rb = uf_find(P, v[i]);
    if (ra == rb) continue;
    if (ra < rb) P[rb] = ra;
    else P[ra] = rb;
    ++counts[bucket[i]];
  }
  free(bucket);
  free(idx);
  free(P);
  return nb;
}
