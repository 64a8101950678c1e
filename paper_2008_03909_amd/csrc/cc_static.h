// Shared host-side state of one static connectivity call.
#pragma once
#include "cc_frontier.h"
#include "cc_internal.h"

namespace cc {

struct StaticArgs {
  cc_ctx* ctx = nullptr;
  hipStream_t s = nullptr;
  int64_t n = 0, m = 0;
  const void* off = nullptr;
  bool o64 = false;
  const int32_t* adj = nullptr;
  const cc_variant* v = nullptr;
  WsLayout L;
  char* ws = nullptr;
  int32_t* P = nullptr;      // parent array == caller's labels_out
  int32_t* count = nullptr;  // n int32 scratch (frequency counts, snapshots)
  int32_t* cand = nullptr;   // thread-bin candidates (also LDD min-member scratch)
  int32_t* big = nullptr;    // wave-bin (front) / block-bin (back) candidates
  int32_t* heavy = nullptr;  // grid-bin candidates / heavy frontier vertices
  long long* hp = nullptr;   // degree prefix of `heavy`
  long long* tsum = nullptr; // tile sums of that prefix
  int64_t hcap = 0;          // capacity of `heavy`
  int64_t heavy_vertices = -1;  // vertices with degree > kHeavyFrontier (-1: not counted yet)
  int2* tree_e = nullptr;    // spanning forest: BFS/LDD tree edge per claimed vertex (nullable)
  int2* hook_e = nullptr;    // spanning forest: union-find edge per hooked root (nullable)
  int64_t* ncomp_user = nullptr;
  bool skip_init = false;    // init (P = identity, counts and scalars cleared) already enqueued
  bool kout_by_xcd = true;   // k-out: each XCD takes its own eighth of the ids (else blocks in id order)
  const int32_t* map_orig = nullptr;  // renumbered CSR: original id of each vertex (output copies it to map_rmin)
  int32_t* map_rmin = nullptr;
  // a call on the first n vertices of a larger graph whose other vertices
  // have no edges: the init still gives all n_parents entries of P a valid
  // parent, and the component count includes the n_parents - n others
  int64_t n_parents = 0;
  int32_t sample_success = 1;
  int32_t sample_rounds = 0;
  int32_t finish_rounds = 0;
  CandLists lists() const { return CandLists{n, cand, big, heavy, hp, ctx->dev->bin_count}; }
};

template <typename I> cc_status sample_bfs(StaticArgs& a);
template <typename I> cc_status sample_ldd(StaticArgs& a);
template <typename I> cc_status finish_sv(StaticArgs& a);
template <typename I> cc_status finish_lt(StaticArgs& a);
template <typename I> cc_status finish_lp(StaticArgs& a);

// Algorithm 1's init on prepared arguments: scalars reset, P = identity,
// frequency counts cleared (the same for every variant).
cc_status static_init(StaticArgs& a);
// The whole static algorithm on prepared arguments (statistics recorded).
cc_status static_run(StaticArgs& a);
// Recompresses the labels, resolves the frequent label (exact counts) and
// builds the degree-binned candidate lists of the vertices outside it.
template <typename I> cc_status prepare_candidates(StaticArgs& a);
// Final compression to canonical labels and the component count.
cc_status output_labels(StaticArgs& a);
// Writes the recorded forest edges (tree_e when given, then hook_e) densely
// to out_u/out_v (and the hook weights to out_w when both are given);
// *num_edges (device) receives the count.  `cnt` holds forest_tiles(len)
// int32.  With orig_of, each endpoint x is written as orig_of[x] (a CSR
// whose vertices were renumbered).
cc_status forest_filter(hipStream_t s, int64_t n, const int2* tree, const int2* hook, const float* hook_w,
                        int32_t* cnt, int32_t* out_u, int32_t* out_v, float* out_w, int64_t* num_edges,
                        const int32_t* orig_of = nullptr);
// After a static run on the first a.n vertices of a renumbered CSR of n
// vertices (a.map_orig set, so the output sweep started each root's
// minimum original id in a.count): labels_out[o] = the smallest original
// id in original vertex o's component, from the labels P in the CSR's
// numbering.  Vertices a.n .. n-1 have empty rows.
cc_status map_back_labels(StaticArgs& a, int64_t n, const int32_t* orig_of, const int32_t* new_of,
                          const int32_t* P, int32_t* labels_out);
int64_t forest_tiles(int64_t len);
// SV / root-based LT rounds over an explicit edge list until nothing changes
// (stream batch inserts with a round-based finish).
cc_status edge_list_rounds(cc_ctx* ctx, hipStream_t s, const cc_variant& v, int64_t n, int32_t* P, int32_t* Q,
                           int32_t* eu, int32_t* ev, const unsigned long long* ecnt, int64_t cap, int32_t* rounds);
// Synchronous read of the context's device scalars into ctx->host.
cc_status pull_scalars(StaticArgs& a);

// Argument checks and workspace carving shared by every static entry point.
cc_status setup_args(StaticArgs& a, cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int o64,
                     const int32_t* adj, const cc_variant* v, void* ws, size_t ws_bytes, int32_t* labels,
                     int64_t* ncomp, void* stream);
// BFS from `source` for at most `level_cap` levels (<= 0: no cap) over the
// workspace bitmaps; reports vertices reached and levels expanded.
template <typename I> cc_status bfs_probe(StaticArgs& a, int32_t source, int level_cap, int64_t* reached,
                                          int32_t* levels);
// Number of vertices with degree > kHeavyFrontier (cached in a).
template <typename I> cc_status count_heavy(StaticArgs& a);
// Degree prefix of a device-counted vertex list: one block when the list is
// known to be short, else the three-launch version.

}  // namespace cc
