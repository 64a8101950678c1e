/*
 * connectit_hip.h -- C ABI of the MI355X (gfx950) connectivity library.
 *
 * Implements the method of "ConnectIt: A Framework for Static and
 * Incremental Parallel Graph Connectivity Algorithms" (Dhulipala, Hong,
 * Shun; arXiv 2008.03909):
 *   - static connectivity (Algorithm 1): init labels, a sampling step
 *     (k-out / BFS / LDD, Section 3.2), IdentifyFrequent, and a finish step
 *     that skips the most frequent sampled component (Section 3.3:
 *     union-find variants, Shiloach-Vishkin, root-based Liu-Tarjan);
 *   - batch-incremental connectivity (Section 3.4 and the appendix
 *     "ConnectIt: Streaming"): Insert(u,v) and IsConnected(u,v) batches.
 *
 * Conventions for every call:
 *   - Vertex ids are int32 in [0, n); n must be in [1, 2^31 - 1].
 *   - Pointers named *_dev or documented as device pointers are device
 *     memory owned by the caller (for example torch tensors); the library
 *     never frees them.  Work is enqueued on `hip_stream` (a hipStream_t;
 *     NULL = the null stream) and is asynchronous unless stated otherwise.
 *   - Labels are canonical: labels_out[v] = the minimum vertex id of v's
 *     connected component, so two runs (any variant) give identical arrays.
 *   - Host-checkable problems (bad sizes, null pointers, an illegal variant,
 *     a too-small workspace) return an error code at once and enqueue
 *     nothing.  Problems only the device can see (an id outside [0, n),
 *     an exceeded round cap) set a device error word; it is reported by the
 *     next call that synchronises and by cc_ctx_sync_status().
 *   - cc_last_error() returns a thread-local detail string for the last
 *     failing call on that thread.
 */
#ifndef CONNECTIT_HIP_H
#define CONNECTIT_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CC_OK = 0,
  CC_EINVAL = -1,       /* bad argument or illegal variant combination */
  CC_ENOMEM = -2,       /* workspace too small or device allocation failed */
  CC_EDEVICE = -3,      /* HIP runtime error or device-detected bad input */
  CC_ELIVELOCK = -4,    /* a round-based phase exceeded its round cap */
  CC_EBUSY = -5,        /* serving loop: request refused by admission */
  CC_EUNSUPPORTED = -6  /* option not built */
} cc_status;

/* Sampling methods, Section 3.2. */
enum { CC_SAMPLE_NONE = 0, CC_SAMPLE_KOUT = 1, CC_SAMPLE_BFS = 2, CC_SAMPLE_LDD = 3 };
/* k-out edge choice: hybrid = first edge + (k-1) uniform picks (the paper's
 * default); afforest = first k edges; pure = k uniform picks. */
enum { CC_KOUT_HYBRID = 0, CC_KOUT_AFFOREST = 1, CC_KOUT_PURE = 2, CC_KOUT_MAXDEG = 3 };
/* maxdeg (appendix "Sampling Schemes", max-degree sampling): pick 0 is the
 * neighbour of largest degree (the first such in row order), then k-1
 * uniform picks as for hybrid. */
/* Finish methods, Section 3.3.  UF-Early and UF-Hooks are the UF-Async
 * relatives of Section 3.3 (any find); LP is label propagation (appendix
 * "Label Propagation"), run as rounds over every candidate edge. */
enum {
  CC_FIN_UF_REM_CAS = 0,
  CC_FIN_UF_ASYNC = 1,
  CC_FIN_SV = 2,
  CC_FIN_LT = 3,
  CC_FIN_UF_EARLY = 4,
  CC_FIN_UF_HOOKS = 5,
  CC_FIN_LP = 6
};
/* Find options (appendix "Find Algorithms"). */
enum { CC_FIND_NAIVE = 0, CC_FIND_ATOMIC_SPLIT = 1, CC_FIND_ATOMIC_HALVE = 2, CC_FIND_COMPRESS = 3 };
/* Splice options of Rem's algorithm (appendix "Splice Algorithms"). */
enum { CC_SPLICE_SPLIT_ONE = 0, CC_SPLICE_HALVE_ONE = 1, CC_SPLICE_ATOMIC = 2 };
/* Liu-Tarjan rule bits (appendix "Liu-Tarjan Algorithms").  Connect kind in
 * the low two bits (Connect, ParentConnect, ExtendedConnect); the other bits
 * add RootUp, FullShortcut (else one Shortcut step per round) and Alter.
 * The appendix's 16 combinations are accepted: the root-based CRSA, PRSA,
 * PRS, CRFA, PRFA, PRF, and the non-root-based CUSA, PUSA, PUS, EUSA, EUS,
 * CUFA, PUFA, PUF, EUFA, EUF (not as stream finishes). */
enum {
  CC_LT_CONNECT = 0,
  CC_LT_PARENT_CONNECT = 1,
  CC_LT_EXTENDED_CONNECT = 2,
  CC_LT_ROOTUP = 4,
  CC_LT_FULL_SHORTCUT = 8,
  CC_LT_ALTER = 16
};
#define CC_LT_CRSA (CC_LT_CONNECT | CC_LT_ROOTUP | CC_LT_ALTER)
#define CC_LT_PRSA (CC_LT_PARENT_CONNECT | CC_LT_ROOTUP | CC_LT_ALTER)
#define CC_LT_PRS (CC_LT_PARENT_CONNECT | CC_LT_ROOTUP)
#define CC_LT_CRFA (CC_LT_CONNECT | CC_LT_ROOTUP | CC_LT_FULL_SHORTCUT | CC_LT_ALTER)
#define CC_LT_PRFA (CC_LT_PARENT_CONNECT | CC_LT_ROOTUP | CC_LT_FULL_SHORTCUT | CC_LT_ALTER)
#define CC_LT_PRF (CC_LT_PARENT_CONNECT | CC_LT_ROOTUP | CC_LT_FULL_SHORTCUT)
#define CC_LT_CUSA (CC_LT_CONNECT | CC_LT_ALTER)
#define CC_LT_PUSA (CC_LT_PARENT_CONNECT | CC_LT_ALTER)
#define CC_LT_PUS (CC_LT_PARENT_CONNECT)
#define CC_LT_EUSA (CC_LT_EXTENDED_CONNECT | CC_LT_ALTER)
#define CC_LT_EUS (CC_LT_EXTENDED_CONNECT)
#define CC_LT_CUFA (CC_LT_CONNECT | CC_LT_FULL_SHORTCUT | CC_LT_ALTER)
#define CC_LT_PUFA (CC_LT_PARENT_CONNECT | CC_LT_FULL_SHORTCUT | CC_LT_ALTER)
#define CC_LT_PUF (CC_LT_PARENT_CONNECT | CC_LT_FULL_SHORTCUT)
#define CC_LT_EUFA (CC_LT_EXTENDED_CONNECT | CC_LT_FULL_SHORTCUT | CC_LT_ALTER)
#define CC_LT_EUF (CC_LT_EXTENDED_CONNECT | CC_LT_FULL_SHORTCUT)

/* One sampling x finish combination (Algorithm 1's sample_opt/finish_opt).
 *  - kout_k >= 1 edges per vertex (paper default 2);
 *  - bfs_tries >= 1 BFS attempts (paper text: 3), success iff the reached
 *    component holds more than n/10 vertices; BFS takes graphs with
 *    m < 2^36 adjacency entries (CC_EINVAL above);
 *  - ldd_beta in (0, 1) (paper default 0.2); ldd_permute must be 0 (the
 *    paper's default ordering; vertex 0 wakes first); LDD takes graphs
 *    with m < 2^36 adjacency entries (CC_EINVAL above);
 *  - find/splice: for UF-Rem-CAS any splice with find in {NAIVE,
 *    ATOMIC_SPLIT, ATOMIC_HALVE}; for UF-Async any find; FIND_COMPRESS with
 *    Rem-CAS (which includes the SpliceAtomic + FindCompress combination of
 *    the paper's counter-example) is rejected with CC_EINVAL;
 *  - seed drives every random draw of the sampler (k-out picks, BFS
 *    sources, LDD shifts); it changes speed, never labels. */
typedef struct {
  int32_t sample;
  int32_t kout_k;
  int32_t kout_mode;
  int32_t bfs_tries;
  float ldd_beta;
  int32_t ldd_permute;
  int32_t finish;
  int32_t find;
  int32_t splice;
  uint32_t lt_rules;
  uint64_t seed;
} cc_variant;

/* Per-call statistics of the last static run on a context (host copy). */
typedef struct {
  int64_t n, m;
  int32_t lmax;              /* skipped sampled component, -1 if none */
  int32_t sample_success;    /* BFS: index of the successful try, else -1; 1 for others */
  int64_t lmax_size;         /* vertices carrying lmax after sampling */
  int64_t candidates;        /* finish vertices (label != lmax and degree > 0) */
  int64_t candidate_edges;   /* adjacency entries the finish visits */
  int32_t sample_rounds;     /* BFS levels / LDD rounds (0 for k-out) */
  int32_t finish_rounds;     /* SV / LT rounds (0 for union-find) */
  int64_t num_components;
  int32_t sample_bottom_up;  /* of sample_rounds, those run bottom-up (speed only) */
  int32_t reserved;
} cc_stats;

typedef struct cc_ctx cc_ctx;
typedef struct cc_stream cc_stream;

/* ---- context -------------------------------------------------------------
 * A context binds a device and owns a few hundred bytes of device state
 * (error word, statistics) allocated here.  Not thread-safe: use one context
 * per host thread.  Returns CC_EDEVICE if the device cannot be used. */
cc_status cc_ctx_create(int device, cc_ctx** out);
void cc_ctx_destroy(cc_ctx* ctx);
/* Synchronises the device and reports (then clears) the device error word. */
cc_status cc_ctx_sync_status(cc_ctx* ctx);
/* Copies the statistics of the last static call (synchronises its stream). */
cc_status cc_last_stats(cc_ctx* ctx, cc_stats* out);
/* When enabled, static calls record HIP events around each phase on the
 * call's stream; cc_phase_times() synchronises and returns the accumulated
 * milliseconds and launch counts per phase since the last reset.  Phase
 * names are stable strings ("init", "sample", "compress_count", "frequent",
 * "compact", "finish", "output", ...). */
cc_status cc_ctx_set_timing(cc_ctx* ctx, int enable);
/* Restricts the recording to the phase named `name` (NULL or "": every
 * phase).  Each recorded event makes the stream wait for the work enqueued
 * before it (about 10 us per event pair here), so timing one phase perturbs
 * a call far less than timing all of them. */
cc_status cc_ctx_set_timing_phase(cc_ctx* ctx, const char* name);
/* Caps the rounds of every round-based phase (BFS levels per try, SV and LT
 * rounds) at `limit` (0 = only the built-in caps); a call that reaches it
 * returns CC_ELIVELOCK, its labels undefined.  A measurement aid for timing
 * many variants without waiting on hopeless ones. */
cc_status cc_ctx_set_round_limit(cc_ctx* ctx, int32_t limit);
int cc_phase_times(cc_ctx* ctx, int max_phases, const char** names, double* total_ms, int64_t* counts);
void cc_phase_times_reset(cc_ctx* ctx);

/* The paper's default: k-out (k = 2, hybrid) + UF-Rem-CAS + SplitAtomicOne
 * + FindNaive, seed 0x5eed. */
cc_status cc_default_variant(cc_variant* out);
/* Validates a variant (same rules as the static calls). */
cc_status cc_check_variant(const cc_variant* v);

/* ---- static connectivity (Algorithm 1) ---------------------------------------
 * Workspace bytes needed by cc_connectivity_csr for (n, m, variant). */
cc_status cc_workspace_bytes(int64_t n, int64_t m, const cc_variant* v, size_t* bytes);

/* labels_out[v] = min id of v's component, for the undirected graph given as
 * a symmetric CSR: offsets (n+1 entries, int64 if offsets_are_64bit else
 * int32; offsets[0] = 0, offsets[n] = m) and adj (m int32 ids).  The CSR
 * must be symmetric (the skip of the frequent component relies on it);
 * rows need not be sorted, but the k-out "first edge" is adj[offsets[v]].
 * Self-loops and duplicates are allowed.  m must fit int32 offsets unless
 * offsets_are_64bit.  The kernels do not range-check offsets or ids: a
 * malformed CSR faults the device instead of returning an error (check
 * untrusted input with cc_validate_csr first).
 * workspace: device buffer of >= cc_workspace_bytes.
 * num_components_dev (nullable): one int64 written on the device.
 * Round-based variants (BFS, LDD, SV, LT) read a 4-byte flag per round and
 * so synchronise hip_stream internally; k-out/none + union-find does not. */
cc_status cc_connectivity_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                              const int32_t* adj, const cc_variant* v, void* workspace, size_t ws_bytes,
                              int32_t* labels_out, int64_t* num_components_dev, void* hip_stream);

/* cc_connectivity_csr on a CSR whose vertices were renumbered (vertex x of
 * the CSR is original vertex orig_of[x]; new_of is the inverse permutation;
 * both device int32[n], e.g. from cc_build_csr_degree_order), with the
 * result in the original numbering: labels_out[o] = the smallest original
 * id in original vertex o's component (the canonical labelling of the
 * original graph, Section 2).  The algorithm runs in the CSR's numbering
 * (k-out's blocks in id order rather than by XCD range), then each
 * component's smallest original id is found (one atomicMin per non-root
 * vertex, aggregated per wave; the frequent component per block) and
 * gathered to the original vertices.  n_active (0..n): the caller's promise
 * that rows n_active .. n-1 are empty (a CSR in decreasing-degree order
 * keeps every isolated vertex there; cc_csr_active_prefix finds the
 * smallest such value; pass n when unknown).  The algorithm then runs on
 * vertices [0, n_active) only, every other vertex being a component of its
 * own; all n labels and the count cover the whole graph.  A broken promise
 * (a non-empty row at or after n_active) is a malformed CSR: the labels are
 * then not defined and the bad-CSR bit of the context's error word is set.
 * With k-out sampling and a union-find finish every access still stays
 * inside the workspace and the caller's arrays (the parent array covers all
 * n vertices, and the arrays sized by n_active lie inside a workspace sized
 * for n); the BFS, LDD,
 * SV, LT and label-propagation variants size their frontier and round
 * arrays by n_active and trust the promise as the static calls trust their
 * CSR (cc_validate_csr on the first n_active rows checks it: every id below
 * n_active).  orig_of and new_of must be inverse
 * permutations of [0, n); they are not checked.  Workspace: device, >=
 * cc_mapped_workspace_bytes (cc_workspace_bytes plus 4n bytes for the
 * labels in the CSR's numbering). */
cc_status cc_mapped_workspace_bytes(int64_t n, int64_t m, const cc_variant* v, size_t* bytes);
cc_status cc_connectivity_csr_mapped(cc_ctx* ctx, int64_t n, int64_t n_active, int64_t m, const void* offsets,
                                     int offsets_are_64bit, const int32_t* adj, const int32_t* orig_of,
                                     const int32_t* new_of, const cc_variant* v, void* workspace, size_t ws_bytes,
                                     int32_t* labels_out, int64_t* num_components_dev, void* hip_stream);
/* *active_dev (device int64) = the smallest x such that rows x .. n-1 of
 * the CSR are all empty (offsets ascending; one lane's binary search on
 * hip_stream).  For a CSR from cc_build_csr_degree_order this is the number
 * of vertices with at least one adjacency entry. */
cc_status cc_csr_active_prefix(int64_t n, const void* offsets, int offsets_are_64bit, int64_t* active_dev,
                               void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as cc_connectivity_csr, with the workspace taken from a fixed device
 * array of cc_noalloc_scratch_bytes() (64 MiB) that the library holds on
 * each device it runs on until the process ends (its address is looked up
 * when a context is created on the device).  The caller still passes the
 * CSR, labels_out and num_components_dev.  A graph whose
 * cc_workspace_bytes exceeds the array returns CC_ENOMEM (with the default
 * variant that is n above about 3 million vertices); nothing is enqueued
 * then.  The call allocates nothing and records no phase events, whatever
 * cc_ctx_set_timing says.  Every call on one device shares that device's
 * array and leaves its contents behind (each call initialises what it
 * reads), so calls that overlap in time on one device -- on different
 * streams, contexts or host threads -- race and must be serialised by the
 * caller. */
size_t cc_noalloc_scratch_bytes(void);
cc_status cc_connectivity_csr_noalloc(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                                      const int32_t* adj, const cc_variant* v, int32_t* labels_out,
                                      int64_t* num_components_dev, void* hip_stream);

/* Sampling step alone (for inspection/tests): writes the sampled partial
 * labelling, each sampled class relabelled to its minimum member, and the
 * frequent label chosen by IdentifyFrequent (or -1).  Same arguments as
 * cc_connectivity_csr; synchronises hip_stream. */
cc_status cc_sample_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                        const int32_t* adj, const cc_variant* v, void* workspace, size_t ws_bytes,
                        int32_t* labels_out, int32_t* lmax_out_host, void* hip_stream);

/* labels_out[v] = min id of v's component for an undirected pair list
 * (u[i], v[i]), i < num_pairs, device int32 arrays (Section 2's edge-list
 * format; self-loops and duplicates allowed, ids must be in [0, n)).  The
 * pairs are first turned into a symmetric deduplicated CSR (as
 * cc_build_csr, int64 offsets when 2*num_pairs >= 2^31) that lives in the
 * workspace, then labelled as by cc_connectivity_csr with variant var.
 * workspace: device buffer of >= cc_coo_workspace_bytes (any alignment).
 * Synchronises hip_stream twice (the sort's size and the edge count).
 * Ids outside [0, n) set the device error word and are dropped. */
cc_status cc_coo_workspace_bytes(int64_t n, int64_t num_pairs, const cc_variant* v, size_t* bytes);
cc_status cc_connectivity_coo(cc_ctx* ctx, int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v,
                              const cc_variant* var, void* workspace, size_t ws_bytes, int32_t* labels_out,
                              int64_t* num_components_dev, void* hip_stream);

/* ---- spanning forest (appendix "ConnectIt: Spanning Forest") --------------------
 * One tree per connected component: edges_u[i], edges_v[i] for
 * i < *num_edges_dev (= n - number of components) are adjacency entries
 * (u, v) of the CSR that together span every component without a cycle.
 * labels_out receives the labels exactly as cc_connectivity_csr would.
 * Every sampler is accepted; BFS and LDD contribute their tree edges, k-out
 * the edges that hooked a union-find root.  The finish must be root-based
 * with CAS hooks: UF-Async (any find) or UF-Rem-CAS with SplitAtomicOne or
 * HalveAtomicOne; SpliceAtomic (which moves non-roots between trees), SV and
 * LT return CC_EUNSUPPORTED.  Which spanning forest comes out depends on the
 * order of concurrent hooks; every one is valid.  edges_u / edges_v: device
 * int32 arrays of at least n entries; num_edges_dev: one device int64.
 * workspace: device buffer of >= cc_forest_workspace_bytes. */
cc_status cc_forest_workspace_bytes(int64_t n, int64_t m, const cc_variant* v, size_t* bytes);
cc_status cc_spanning_forest_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                                 const int32_t* adj, const cc_variant* v, void* workspace, size_t ws_bytes,
                                 int32_t* labels_out, int32_t* edges_u, int32_t* edges_v, int64_t* num_edges_dev,
                                 void* hip_stream);
/* The spanning forest of a renumbered CSR (orig_of / new_of and n_active as
 * for cc_connectivity_csr_mapped), reported in the original numbering: each
 * forest edge (edges_u[i], edges_v[i]) is a pair of original ids, and
 * labels_out[o] is the smallest original id in original vertex o's
 * component.  The algorithm runs on vertices [0, n_active); the others have
 * no edges and add none.  Variants as for cc_spanning_forest_csr.
 * workspace: device buffer of >= cc_forest_mapped_workspace_bytes
 * (cc_forest_workspace_bytes plus 4n bytes for the labels in the CSR's
 * numbering). */
cc_status cc_forest_mapped_workspace_bytes(int64_t n, int64_t m, const cc_variant* v, size_t* bytes);
cc_status cc_spanning_forest_csr_mapped(cc_ctx* ctx, int64_t n, int64_t n_active, int64_t m, const void* offsets,
                                        int offsets_are_64bit, const int32_t* adj, const int32_t* orig_of,
                                        const int32_t* new_of, const cc_variant* v, void* workspace, size_t ws_bytes,
                                        int32_t* labels_out, int32_t* edges_u, int32_t* edges_v,
                                        int64_t* num_edges_dev, void* hip_stream);

/* ---- approximate minimum spanning forest (Section 5.1, AMSF) -------------------
 * weights[j] > 0 is the weight of adjacency entry j of the symmetric CSR
 * (device float array of m entries); both orientations of an edge must carry
 * the same weight.  With W_min the smallest weight, the edges are bucketed
 * by thresholds t_0 = W_min, t_{i+1} = t_i * (1 + epsilon) computed in
 * double and rounded down to float (so every bucket [t_i, t_{i+1}) spans a
 * ratio of at most 1 + epsilon), and buckets are taken in increasing order:
 * each adds a spanning forest of its edges over the components of the
 * buckets before it.  The result is a spanning forest whose weight is at
 * most (1 + epsilon) times the minimum; the number of its edges in each
 * bucket is the same for every such forest.
 *
 * The first buckets, holding about light_fraction of the entries (estimated
 * from a sample of the weights), are extracted once into a bucket-sorted
 * edge list; every later bucket is a round over the rows of the vertices
 * outside the largest component of the labelling so far (the paper's
 * sampled no-filter variant, AMSF-NF-S).  light_fraction = 0 runs every
 * bucket that way.  Union-find is UF-Rem-CAS with SplitAtomicOne and
 * FindNaive, as in the paper's experiments.
 *
 * Outputs: edges_u / edges_v / edges_w (device, at least n entries each;
 * edges_w nullable) receive *num_edges_dev (device int64) forest edges;
 * labels_out receives the canonical component labels (min id);
 * weight_dev (nullable, device double) the forest's total weight.
 * Errors: epsilon outside [2^-20, 2^20], light_fraction outside [0, 1] or
 * bucket counts above 4096 (the weight range spans more than
 * (1 + epsilon)^4096) return CC_EINVAL; a weight that is not finite and > 0
 * returns CC_EINVAL after the first pass.  The call synchronises hip_stream
 * twice (after the light buckets are counted, and after the candidate lists
 * of the later rounds are built).
 * workspace: device buffer of >= cc_amsf_workspace_bytes. */
typedef struct {
  float epsilon;         /* bucket ratio - 1 (the paper's experiments: 0.25) */
  float light_fraction;  /* share of entries handled from the bucket-sorted list (default 0.4) */
  uint64_t seed;         /* weight sample used to pick the light buckets */
} cc_amsf_options;
cc_status cc_amsf_default_options(cc_amsf_options* out);
cc_status cc_amsf_workspace_bytes(int64_t n, int64_t m, const cc_amsf_options* opt, size_t* bytes);
cc_status cc_amsf_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                      const int32_t* adj, const float* weights, const cc_amsf_options* opt, void* workspace,
                      size_t ws_bytes, int32_t* labels_out, int32_t* edges_u, int32_t* edges_v, float* edges_w,
                      int64_t* num_edges_dev, double* weight_dev, void* hip_stream);
/* cc_amsf_csr on a renumbered CSR (orig_of / new_of and n_active as for
 * cc_connectivity_csr_mapped; weights[j] is the weight of the CSR's
 * adjacency entry j), reported in the original numbering: forest edges as
 * pairs of original ids, labels_out[o] the smallest original id in o's
 * component.  The unions run on vertices [0, n_active); every row of the
 * CSR is still scanned once to cut the adjacency into tiles.  workspace: >=
 * cc_amsf_mapped_workspace_bytes (cc_amsf_workspace_bytes plus 4n bytes for
 * the labels in the CSR's numbering). */
cc_status cc_amsf_mapped_workspace_bytes(int64_t n, int64_t m, const cc_amsf_options* opt, size_t* bytes);
cc_status cc_amsf_csr_mapped(cc_ctx* ctx, int64_t n, int64_t n_active, int64_t m, const void* offsets,
                             int offsets_are_64bit, const int32_t* adj, const int32_t* orig_of, const int32_t* new_of,
                             const float* weights, const cc_amsf_options* opt, void* workspace, size_t ws_bytes,
                             int32_t* labels_out, int32_t* edges_u, int32_t* edges_v, float* edges_w,
                             int64_t* num_edges_dev, double* weight_dev, void* hip_stream);

/* ---- ingest: undirected pair list -> symmetric CSR (Section 2 formats) -------
 * Output: both orientations of every pair with u != v, rows sorted
 * ascending, duplicates removed iff dedup != 0.  adj_out needs capacity
 * 2*num_pairs; offsets_out gets n+1 entries (int64 if offsets_64bit).  The
 * edge count m is written to *m_dev (device int64).  Ids outside [0, n) set
 * the device error word and are dropped.  The workspace (at least
 * cc_csr_workspace_bytes) must be 256-byte aligned.  Synchronises hip_stream
 * once (to size the sort). */
cc_status cc_csr_workspace_bytes(int64_t n, int64_t num_pairs, size_t* bytes);
cc_status cc_build_csr(cc_ctx* ctx, int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v, int dedup,
                       void* workspace, size_t ws_bytes, void* offsets_out, int offsets_64bit, int32_t* adj_out,
                       int64_t* m_dev, void* hip_stream);

/* The same CSR with its vertices renumbered by decreasing degree (the
 * degree of cc_build_csr's output, ties by smaller id; a degree above
 * 2^b - 1, b = bits of n - 1, counts as 2^b - 1): vertex x of the output is
 * original vertex orig_of[x], and new_of[o] is the new number of original
 * vertex o (both device int32[n], written by the call).  A layout choice
 * made at ingest: on power-law graphs the hubs' parent entries then share
 * a few cache lines and the k-out picks of low-degree vertices land on them.
 * Use the result with cc_connectivity_csr_mapped to get labels in the
 * original numbering.  Ids outside [0, n) are reported as by cc_build_csr.
 * Workspace: device, 256-byte aligned, >= cc_csr_degree_order_workspace_bytes.
 * Synchronises hip_stream twice. */
cc_status cc_csr_degree_order_workspace_bytes(int64_t n, int64_t num_pairs, size_t* bytes);
cc_status cc_build_csr_degree_order(cc_ctx* ctx, int64_t n, int64_t num_pairs, const int32_t* u, const int32_t* v,
                                    int dedup, void* workspace, size_t ws_bytes, void* offsets_out, int offsets_64bit,
                                    int32_t* adj_out, int64_t* m_dev, int32_t* orig_of, int32_t* new_of,
                                    void* hip_stream);

/* ---- CSR validator (debug aid) ----------------------------------------------
 * The static calls trust their CSR: they index the parent array with
 * adjacency ids and the adjacency with offsets without range checks, so a
 * malformed CSR is a GPU memory fault there, not an error code; and the skip
 * of the most frequent sampled component (Section 3.1) is only correct on a
 * symmetric graph (appendix "Correctness for Sampling Algorithms").
 * cc_validate_csr checks a CSR before use:
 *   CC_CSR_OFFSET0     offsets[0] != 0;
 *   CC_CSR_OFFSETN     offsets[n] != m;
 *   CC_CSR_MONOTONE    some row has offsets[v] > offsets[v+1], or a bound
 *                      outside [0, m] (its entries are then not read);
 *   CC_CSR_ID_RANGE    some adjacency id outside [0, n);
 *   CC_CSR_ASYMMETRIC  (check_symmetric != 0, only run when the checks above
 *                      pass) some entry (v, w) has no entry (w, v).  With
 *                      every row ascending this is exact (a binary search in
 *                      row w per entry; bad_entries counts the entries
 *                      without a reverse); otherwise the multisets {(v, w)}
 *                      and {(w, v)} are compared by a 64-bit hash sum, so a
 *                      symmetric CSR always passes, an asymmetric one fails
 *                      but for a 64-bit hash coincidence, and a pair stored
 *                      more often in one direction than the other counts as
 *                      asymmetric.
 * Inputs as for cc_connectivity_csr (device offsets and adj); report is a
 * host struct.  Returns CC_OK for a valid CSR and CC_EDEVICE when a check
 * failed (report says which); host-checkable argument errors give
 * CC_EINVAL.  The device-side checks set the context's error word (bad id,
 * malformed CSR) and the call clears it again after reading it; an error
 * word left by an earlier call is returned first, without validating.
 * Synchronises the device (once) and hip_stream (twice or three times);
 * allocates nothing. */
enum { CC_CSR_OFFSET0 = 1, CC_CSR_OFFSETN = 2, CC_CSR_MONOTONE = 4, CC_CSR_ID_RANGE = 8, CC_CSR_ASYMMETRIC = 16 };
typedef struct {
  uint32_t failed;          /* CC_CSR_* bits of the checks that failed (0: valid) */
  int32_t rows_sorted;      /* 1 iff every well-formed row is ascending */
  int32_t symmetry_checked; /* 0 not checked, 1 exact (ascending rows), 2 hash of multisets */
  int32_t reserved;
  int64_t bad_entries;      /* ids out of range, or (exact check) entries without a reverse */
  int64_t first_bad_row;    /* smallest row where a check failed, -1 if none or unknown */
} cc_csr_report;
cc_status cc_validate_csr(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                          const int32_t* adj, int check_symmetric, cc_csr_report* report, void* hip_stream);

/* ---- batch-incremental connectivity (Section 3.4 "Streaming") ---------------
 * A cc_stream owns an n x int32 parent array on the device (allocated by
 * cc_stream_create, freed by cc_stream_destroy), starting from the empty
 * graph.  Every finish is accepted; it decides the streaming type (Section
 * 3.4): type 1 = UF-Async (any find) and UF-Rem-CAS with SplitAtomicOne or
 * HalveAtomicOne (inserts and queries may run concurrently); type 2 = SV
 * and the root-based LT variants (inserts in synchronous rounds over the
 * batch; these streams also own an n x int32 snapshot and an edge list of
 * 2^22 pairs, allocated here, and insert a larger batch as consecutive
 * parts of that size, so no insert allocates); type 3 =
 * UF-Rem-CAS with SpliceAtomic (phase-concurrent).  NULL v: UF-Async with
 * FindNaive.  On one cc_stream, every batch reflects exactly the batches
 * enqueued before it in stream order.  Type-2 inserts synchronise
 * hip_stream once per round. */
cc_status cc_stream_create(cc_ctx* ctx, int64_t n, const cc_variant* v, cc_stream** out);
void cc_stream_destroy(cc_stream* s);
/* Initialize(G): the static algorithm on a symmetric CSR, result kept as the
 * stream's state.  workspace as for cc_connectivity_csr. */
cc_status cc_stream_init_csr(cc_stream* s, int64_t m, const void* offsets, int offsets_are_64bit,
                             const int32_t* adj, void* workspace, size_t ws_bytes, void* hip_stream);
/* Insert(u[i], v[i]) for i < k (device arrays). */
cc_status cc_insert_batch(cc_stream* s, int64_t k, const int32_t* u, const int32_t* v, void* hip_stream);
/* out[i] = IsConnected(a[i], b[i]) as 0/1 bytes (device arrays). */
cc_status cc_query_batch(cc_stream* s, int64_t q, const int32_t* a, const int32_t* b, uint8_t* out,
                         void* hip_stream);
/* One mixed batch (the streaming appendix's ProcessBatch): for i < k,
 * kind[i] == 0 is Insert(u[i], v[i]) and any other kind is IsConnected(u[i],
 * v[i]), answered in out[i] (0/1; 0 for inserts); all device arrays.  The
 * answers are linearizable with respect to the batch's inserts: a query
 * answers 1 if its endpoints were connected before the batch and 0 if they
 * are not connected after it.  Type 1 runs inserts and queries together in
 * one kernel (queries are Jayanti-Tarjan SameSet); types 2 and 3 run the
 * inserts first, then the queries.  Ids outside [0, n) set the error word
 * and the operation is skipped (answer 0). */
cc_status cc_process_batch(cc_stream* s, int64_t k, const uint8_t* kind, const int32_t* u, const int32_t* v,
                           uint8_t* out, void* hip_stream);
/* The stream's type (1, 2 or 3 as above; 0 for NULL). */
int32_t cc_stream_type(const cc_stream* s);
/* Canonical labels of the current state (labels_out: n int32 device). */
cc_status cc_stream_labels(cc_stream* s, int32_t* labels_out, int64_t* num_components_dev, void* hip_stream);
/* Synchronises and reports (then clears) the stream's device error word. */
cc_status cc_stream_sync_status(cc_stream* s);

/* ---- serving loop (continuous batching over one device state) -------------------
 * A cc_server owns a device union-find state for n vertices, a device request
 * pool of budget_bytes, num_streams HIP streams (1..16) and at most
 * max_inflight requests on the device.  Requests are admitted in arrival
 * order when a slot is free and, for requests that are copied (below), their
 * bytes (8 per pair, plus 1 per query pair) fit in the pool; every query
 * answers against exactly the inserts that arrived before it
 * (the batch-incremental semantics of the streaming appendix, arrival order =
 * batch order; Section 3.4).  Two modes:
 *   - v NULL or UF-Async with FindNaive (stamped mode, the type-1 setting of
 *     Section 3.4): consecutive insert requests with no query between them
 *     form a numbered insert phase and run concurrently; each link records
 *     its phase number (the state is n 64-bit words); a phase starts after
 *     the previous one completed.  A query runs once the inserts that arrived
 *     before it have completed and reads only links of those phases, so it
 *     overlaps the insert requests that arrive after it.  Inserts shorten
 *     paths (path splitting) only where no query in flight can tell: two
 *     consecutive links of one phase, or of phases that no such query
 *     separates;
 *   - any other variant (barrier mode): the server owns a cc_stream of that
 *     variant; consecutive requests of one type run concurrently and each
 *     change between inserts and queries is ordered by a barrier event.
 * The server's host state is bounded: completed requests are freed, HIP
 * events are reused, and cc_server_request_info keeps the outcome of the
 * 65,536 most recent completions (older ids return CC_EINVAL).  Single host
 * thread.  Payloads: when a request's arrays (and out, for a query) are
 * host memory mapped into the device's address space (pinned, e.g.
 * hipHostMalloc or a pinned torch tensor; checked with
 * hipPointerGetAttributes over each whole range), the kernels read the pairs
 * and write the 0/1 answers in place and the request takes no pool bytes;
 * otherwise the server copies the pairs into the pool on a copy stream of its
 * own and copies the answers back.  Either way every array must stay valid
 * and unmodified until its request completes.  A copied request larger than
 * the budget returns CC_EBUSY.  Ids outside [0, n) set the state's
 * error word (reported by cc_server_poll with wait_all) and are skipped
 * (queries answer 0).  Times are seconds on the server's steady clock
 * (cc_server_clock); arrival < 0 means "now". */
typedef struct cc_server cc_server;
cc_status cc_server_create(cc_ctx* ctx, int64_t n, const cc_variant* v, int64_t budget_bytes, int num_streams,
                           int max_inflight, cc_server** out);
void cc_server_destroy(cc_server* s);
double cc_server_clock(cc_server* s);
/* 1 if the server runs in stamped mode (queries overlap later inserts). */
int32_t cc_server_stamped(const cc_server* s);
/* HIP events the server has created so far (they are reused; bounded by the
 * requests in flight, not by the requests served). */
int64_t cc_server_event_count(const cc_server* s);
cc_status cc_server_submit_insert(cc_server* s, int64_t k, const int32_t* u_host, const int32_t* v_host,
                                  double arrival, int64_t* id);
cc_status cc_server_submit_query(cc_server* s, int64_t q, const int32_t* a_host, const int32_t* b_host,
                                 uint8_t* out_host, double arrival, int64_t* id);
/* Retires finished requests and admits pending ones; wait_all != 0 blocks
 * until every submitted request has completed, then reports (and clears) the
 * state's device error word. */
cc_status cc_server_poll(cc_server* s, int wait_all);
/* Replays a trace in real time: request i (type 0 insert / 1 query) arrives
 * arrival_s[i] seconds after the call and carries pairs [start[i],
 * start[i]+len[i]) of a/b (host arrays); query answers go to out at the same
 * positions; latency_s[i] = completion - arrival.  Returns after all finish. */
cc_status cc_server_run_trace(cc_server* s, int64_t count, const int32_t* type, const double* arrival_s,
                              const int64_t* start, const int64_t* len, const int32_t* a, const int32_t* b,
                              uint8_t* out, double* latency_s);
cc_status cc_server_request_info(cc_server* s, int64_t id, int* done, double* latency_s);
/* Labels of the state after every submitted request (waits for all). */
cc_status cc_server_labels(cc_server* s, int32_t* labels_out, int64_t* num_components_dev, void* hip_stream);
/* Bytes of the device pool currently held by admitted requests. */
int64_t cc_server_pool_used(cc_server* s);

/* ---- learned variant selector ---------------------------------------------------
 * Not part of the paper's method: it only chooses among its variants, so it
 * changes speed, never labels.  Model: 16 features -> 64 -> 64 -> K (ReLU),
 * parameters packed as BF16 [W1 16x64 | b1 64 | W2 64x64 | b2 64 | W3 64xK |
 * b3 K] (row-major, input index first), inputs and hidden activations
 * rounded to BF16, FP32 accumulation, FP32 outputs (predicted log-time of
 * each arm relative to the best).  1 <= K <= 128.  All arrays are device
 * memory unless named *_host. */
int64_t cc_mlp_param_count(int32_t num_arms);
/* Y[B x K] = MLP(X[B x 16]); cache (nullable, B x 256 floats) keeps the
 * hidden pre-/post-activations for cc_mlp_backward. */
cc_status cc_mlp_forward(const uint16_t* params, int32_t K, int32_t B, const float* X, float* Y, float* cache,
                         void* hip_stream);
/* grads (FP32, parameter packing) = d/dparams of mean((Y - T)^2) over the
 * B x K entries, BF16 rounding treated as identity; scratch: 4*B*64 floats;
 * loss (nullable, device float) receives the loss. */
cc_status cc_mlp_backward(const uint16_t* params, int32_t K, int32_t B, const float* X, const float* cache,
                          const float* Y, const float* T, float* grads, float* scratch, float* loss,
                          void* hip_stream);
/* One Adam step (step >= 1) on FP32 master weights; params gets their BF16 copy. */
cc_status cc_mlp_adam(float* master, uint16_t* params, const float* grads, float* m1, float* m2, int64_t count,
                      float lr, float beta1, float beta2, float eps, int32_t step, void* hip_stream);
/* dst = BF16(src), round to nearest even. */
cc_status cc_mlp_pack_bf16(const float* src, uint16_t* dst, int64_t count, void* hip_stream);
/* The 16 features of a symmetric CSR: degree statistics (log2 n,
 * log2(m+1), m/n, coefficient of variation, max/mean, fractions of degree 0,
 * 1 and <= 2, skewness, [m/n < 3], log2(max degree + 1)); statistics of
 * 4096 seeded vertex draws (fraction whose first neighbour id is smaller,
 * mean log-distance to it, mean log-degree of it); and 16 BFS probes from
 * seeded sources, each expanding whole levels within 4 levels and 1024
 * scanned adjacency entries (mean levels expanded, mean fraction of
 * vertices reached).  The exact definitions are in the selector source.
 * workspace as for cc_connectivity_csr with the default variant.
 * Synchronises hip_stream. */
cc_status cc_graph_features(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                            const int32_t* adj, void* workspace, size_t ws_bytes, float* features_host,
                            void* hip_stream);
/* The arm the model predicts fastest, without running it: features,
 * normalisation and forward pass as in cc_connectivity_auto, then
 * out_host = arms[argmin].  params_dev NULL gives the default variant
 * (chosen -1).  workspace as for cc_connectivity_auto.  Synchronises
 * hip_stream once. */
cc_status cc_select_variant(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                            const int32_t* adj, const uint16_t* params_dev, int32_t K, const cc_variant* arms,
                            const float* norm_host, void* workspace, size_t ws_bytes, cc_variant* out_host,
                            int32_t* chosen_host, float* features_host, void* hip_stream);
/* Small-graph gate of cc_connectivity_auto: with a model, graphs of fewer
 * than min_vertices vertices skip the features and the forward pass and run
 * arms[arm] (a choice learned from the training corpus), because the
 * selector's fixed cost there exceeds what choosing saves; chosen_host then
 * reports `arm` and features_host NaN.  min_vertices = 0 turns the gate off
 * (the default).  Applies to calls on this context. */
cc_status cc_ctx_set_selector_gate(cc_ctx* ctx, int64_t min_vertices, int32_t arm);
/* Static connectivity with the arm the model predicts fastest: the 16
 * features, x = (f - norm_host[0:16]) / norm_host[16:32], the forward pass
 * and the argmin over the K arms (host array of variants) all run on the
 * device and are read back with one synchronisation, then the chosen arm
 * runs as cc_connectivity_csr.  Algorithm 1's init (labels_out = identity,
 * counts cleared), the same for every arm, is enqueued before the host
 * waits, so it runs during the wait.  params_dev NULL runs the default
 * variant.
 * chosen_host (nullable) gets the arm index (-1 for the default);
 * features_host (nullable) gets the 16 features.  workspace: at least the
 * largest cc_workspace_bytes over the arms and the default. */
cc_status cc_connectivity_auto(cc_ctx* ctx, int64_t n, int64_t m, const void* offsets, int offsets_are_64bit,
                               const int32_t* adj, const uint16_t* params_dev, int32_t K, const cc_variant* arms,
                               const float* norm_host, void* workspace, size_t ws_bytes, int32_t* labels_out,
                               int64_t* num_components_dev, int32_t* chosen_host, float* features_host,
                               void* hip_stream);

/* ---- calibration (measurement aids) ------------------------------------------
 * Roofline anchors for the kernels above; they compute nothing the method
 * needs.  cc_calib_copy: dst = src for `bytes` bytes (both 16-byte aligned,
 * bytes a multiple of 16) -- the attainable streaming bandwidth.
 * cc_calib_edges: the paper's MapEdges (vals == NULL: out[v] = number of
 * adjacency entries read for v) or GatherEdges (out[v] = sum over v's
 * neighbours w of vals[w], int32 wrap-around), the practical lower bounds of
 * the appendix "Comparison with MapEdges and GatherEdges".  out: n int32;
 * workspace: device bytes >= cc_calib_workspace_bytes(m). */
cc_status cc_calib_copy(const void* src, void* dst, size_t bytes, void* hip_stream);
cc_status cc_calib_workspace_bytes(int64_t m, size_t* bytes);
cc_status cc_calib_edges(int64_t n, int64_t m, const void* offsets, int offsets_are_64bit, const int32_t* adj,
                         const int32_t* vals, int32_t* out, void* workspace, size_t ws_bytes, void* hip_stream);

const char* cc_status_string(cc_status st);
const char* cc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CONNECTIT_HIP_H */
