// Host-side internals shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "connectit_hip.h"

namespace cc {

// Device-resident per-context scalars.  Kernels update these; the host reads
// them back only where a round loop needs a decision or on request.
struct DevScalars {
  uint32_t error;          // bit 0: id out of range; bit 1: round cap; bit 2: bad CSR
  uint32_t changed;        // round-based finishes: set when a round changed a parent
  unsigned long long lmax_key;  // (count << 32) | ~label, max-reduced by IdentifyFrequent
  int32_t lmax;            // resolved frequent label (-1: none)
  int32_t bfs_min;         // minimum vertex reached by the current BFS
  int32_t bin_count[4];    // candidate bins: thread / wave / block / (unused)
  long long cand_edges;    // adjacency entries owned by candidates
  long long num_components;
  long long lmax_size;
  uint32_t qcount[2];      // frontier queue lengths (ping-pong)
  long long frontier_edges;    // degree sum of the next frontier
  uint32_t bfs_mode;       // BFS level direction: 0 top-down, 1 bottom-up, 2 finished
  int32_t bfs_level;       // BFS levels expanded
  long long reached;       // vertices reached by the current BFS (follows bfs_mode/bfs_level: read together)
  long long seen_edges;    // BFS: degree sum of every frontier so far
  unsigned long long heavy_count;  // vertices with degree above the frontier threshold
  unsigned long long heavy_pack;   // LDD: heavy frontier rows (high 28 bits) and their edges (low 36)
  uint32_t flag2;          // spare flag for sub-rounds (full shortcut)
  int32_t hcount;          // k-out max-degree: rows long enough for a wave each
  long long ldd_fe[2];     // LDD: degree sum of the frontier being built in queue 0 / 1
  long long ldd_seen;      // LDD: degree sum of every frontier expanded so far
  int32_t bu_rounds;       // BFS levels / LDD rounds run bottom-up in this call
  uint32_t pad[5];         // pad[0]: LDD minimum draw
  // CSR validator (cc_validate_csr): failed checks (CC_CSR_* bits), bad
  // entries, smallest failing row, unsorted-row flag, symmetry fingerprint
  uint32_t csr_failed;
  uint32_t csr_unsorted;
  long long csr_bad;
  long long csr_first;
  unsigned long long csr_fp;
  int32_t fbin[2][4];      // label propagation: bin lengths of the frontier lists (double-buffered)
  long long map_tail;      // renumbered CSR: first vertex from which every row is empty
};

enum : uint32_t { kErrBadId = 1u, kErrRoundCap = 2u, kErrBadCsr = 4u };

struct PhaseRec {
  const char* name;
  hipEvent_t a, b;
};

}  // namespace cc

struct cc_ctx {
  int device = 0;
  cc::DevScalars* dev = nullptr;     // device copy
  cc::DevScalars* host = nullptr;    // pinned host mirror
  float* sel_host = nullptr;         // pinned, coherent: selector features + choice
  float* sel_dev = nullptr;          // the same memory as the device addresses it
  uint32_t sel_seq = 0;              // sequence number of the last selector call
  unsigned char* ring_host = nullptr;  // pinned: BFS progress snapshots (2 x 16 bytes)
  hipEvent_t ring_ev[2] = {nullptr, nullptr};  // marks each snapshot's copy (created with the context)
  void* amsf_host = nullptr;         // pinned: bucket histogram of the last AMSF call (allocated on first use)
  void* noalloc_scratch = nullptr;   // device address of this device's no-allocation workspace array
  cc_stats last{};
  int round_limit = 0;  // 0: the built-in caps only
  int64_t gate_vertices = 0;  // selector: graphs below this many vertices skip the model (0: never)
  int32_t gate_arm = -1;      // the arm they run instead
  // phase timing
  int timing = 0;
  std::string timing_only;                  // non-empty: record only the phase of this name
  std::vector<cc::PhaseRec> pending;        // events of calls not yet harvested
  std::vector<hipEvent_t> event_pool;
  std::vector<std::string> phase_names;
  std::vector<double> phase_ms;
  std::vector<int64_t> phase_cnt;
};

namespace cc {

// thread-local error message
void set_error(const char* fmt, ...);
cc_status fail(cc_status st, const char* fmt, ...);

#define CC_HIP(expr)                                                                     \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess)                                                                \
      return ::cc::fail(CC_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), \
                        __FILE__, __LINE__);                                             \
  } while (0)

#define CC_LAUNCH_CHECK()                                                                          \
  do {                                                                                             \
    hipError_t _e = hipGetLastError();                                                             \
    if (_e != hipSuccess)                                                                          \
      return ::cc::fail(CC_EDEVICE, "kernel launch failed: %s (%s:%d)", hipGetErrorString(_e), __FILE__, \
                        __LINE__);                                                                 \
  } while (0)

// Phase timing: records an event pair around a phase when ctx->timing is on.
struct PhaseScope {
  cc_ctx* ctx;
  hipStream_t s;
  const char* name;
  hipEvent_t a = nullptr;
  PhaseScope(cc_ctx* c, hipStream_t st, const char* nm);
  ~PhaseScope();
};

inline int64_t div_up(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline unsigned grid_for(int64_t work, int block, int64_t cap = (int64_t)1 << 20) {
  int64_t g = div_up(work > 0 ? work : 1, block);
  return (unsigned)(g < cap ? g : cap);
}
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// XCD-aware vertex sweeps.  The device hands consecutive blocks of a launch
// to its 8 XCDs in turn (block b to XCD b mod 8), and each XCD has its own
// L2.  In a launch whose block count is a multiple of 8, xcd_sweep lets the
// blocks of XCD x walk the x-th eighth of [0, n) in order, so the vertices
// one XCD works on at a time are neighbours in id order and share that
// XCD's cache lines; any other block count gets a plain grid-stride sweep.
// A different dispatch order only costs speed.
constexpr int kXcds = 8;
inline unsigned xcd_grid(int64_t work, int block, int64_t cap) {
  const int64_t g = grid_for(work, block, cap);
  return (unsigned)(g >= kXcds ? g / kXcds * kXcds : g);
}

// Workspace layout of a static call.
struct WsLayout {
  size_t count = 0;       // n int32: IdentifyFrequent counts / SV prev / LT snapshot
  size_t cand = 0;        // n int32: thread-bin candidates
  size_t big = 0;         // n int32: wave-bin (front) and block-bin (back) candidates
  size_t bits = 0;        // 3 bitmaps of n bits (BFS / LDD)
  size_t queue = 0;       // 2 * n int32 frontier queues
  size_t edges = 0;       // LT with Alter: 2 * m int32 (edge list)
  size_t hist = 0;        // LDD start-round histogram
  size_t seg = 0;         // compaction: per-segment counts and edge sums
  size_t heavy = 0;       // grid-bin vertex list and its degree prefix
  size_t mlp = 0;         // selector: one feature row and its scores
  size_t total = 0;
};
WsLayout ws_layout(int64_t n, int64_t m, const cc_variant* v);
cc_status check_variant(const cc_variant* v, bool for_stream);

}  // namespace cc
