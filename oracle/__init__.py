"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the device
library: the C half (``oracle.c``) is compiled by gcc into ``liboracle.so``;
the numpy half is written here from the definitions in the ConnectIt paper
(arXiv 2008.03909).  Each function names the passage it follows.

Pinning: every function here is checked by ``tests/test_oracle_pins.py``
against closed forms, brute force, invariants and the paper's worked
example, not against itself.  ``identify_frequent`` and the MLP reference
are pinned by hand-computed fixtures and finite differences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError(f"{_SO} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(_SO)
        i64 = ctypes.c_int64
        lib.oracle_csr_build.argtypes = [i64, i64, _i32p, _i32p, ctypes.c_int, _i64p, _i32p]
        lib.oracle_csr_build.restype = i64
        lib.oracle_bfs_cc.argtypes = [i64, _i64p, _i32p, _i32p]
        lib.oracle_bfs_cc.restype = i64
        lib.oracle_uf_cc.argtypes = [i64, i64, _i32p, _i32p, _i32p]
        lib.oracle_uf_cc.restype = i64
        lib.oracle_closure_cc.argtypes = [i64, i64, _i32p, _i32p, _i32p]
        lib.oracle_closure_cc.restype = i64
        lib.oracle_uf_init.argtypes = [i64, _i32p]
        lib.oracle_uf_insert.argtypes = [i64, _i32p, i64, _i32p, _i32p]
        lib.oracle_uf_query.argtypes = [i64, _i32p, i64, _i32p, _i32p, _u8p]
        lib.oracle_uf_labels.argtypes = [i64, _i32p, _i32p]
        lib.oracle_uf_labels.restype = i64
        lib.oracle_kout_sample.argtypes = [i64, _i64p, _i32p, ctypes.c_int32, ctypes.c_uint64, _i32p]
        lib.oracle_kout_sample.restype = i64
        lib.oracle_bfs_sample.argtypes = [i64, _i64p, _i32p, ctypes.c_int32, ctypes.c_uint64, _i32p]
        lib.oracle_bfs_sample.restype = i64
        lib.oracle_splitmix_out.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_splitmix_out.restype = ctypes.c_uint64
        lib.oracle_bfs_levels.argtypes = [i64, _i64p, _i32p, ctypes.c_int32, ctypes.c_int32, _i32p]
        lib.oracle_bfs_levels.restype = i64
        lib.oracle_bfs_budget.argtypes = [i64, _i64p, _i32p, ctypes.c_int32, ctypes.c_int32, i64, _i32p]
        lib.oracle_bfs_budget.restype = i64
        lib.oracle_forest_check.argtypes = [i64, _i64p, _i32p, _i32p, i64, _i32p, _i32p]
        lib.oracle_forest_check.restype = i64
        lib.oracle_msf_weight.argtypes = [i64, i64, _i32p, _i32p, ctypes.POINTER(ctypes.c_double), _i64p]
        lib.oracle_msf_weight.restype = ctypes.c_double
        lib.oracle_amsf_buckets.argtypes = [i64, i64, _i32p, _i32p, ctypes.POINTER(ctypes.c_float),
                                            ctypes.c_double, ctypes.c_int32, ctypes.POINTER(ctypes.c_float), _i64p]
        lib.oracle_amsf_buckets.restype = ctypes.c_int32
        lib.oracle_kout_sample_mode.argtypes = [i64, _i64p, _i32p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                                _i32p]
        lib.oracle_kout_sample_mode.restype = i64
        _lib = lib
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _p32(a):
    return a.ctypes.data_as(_i32p)


def _p64(a):
    return a.ctypes.data_as(_i64p)


# ---- adjacency ------------------------------------------------------------

def csr_build(n: int, u, v, dedup: bool = True):
    """CSR of the undirected pair list (Section 2, "Graph Notation and Formats").

    Both orientations of every non-loop pair; rows ascending; with ``dedup``
    one copy of each directed edge.  Returns (offsets int64[n+1], adj int32[m]).
    """
    u, v = _c(u, np.int32), _c(v, np.int32)
    offsets = np.zeros(n + 1, np.int64)
    adj = np.empty(max(2 * u.shape[0], 1), np.int32)
    m = _load().oracle_csr_build(n, u.shape[0], _p32(u), _p32(v), int(dedup), _p64(offsets), _p32(adj))
    return offsets, adj[:m].copy()


# ---- connectivity labelling: label[v] = min id reachable from v -------------

def bfs_cc(n: int, offsets, adj):
    """Sequential BFS sweep over a CSR (Section 2 connectivity labelling)."""
    offsets, adj = _c(offsets, np.int64), _c(adj, np.int32)
    lab = np.empty(n, np.int32)
    c = _load().oracle_bfs_cc(n, _p64(offsets), _p32(adj) if adj.size else _p32(np.zeros(1, np.int32)), _p32(lab))
    return lab, int(c)


def uf_cc(n: int, u, v):
    """Sequential union-find over a pair list (larger root linked under smaller)."""
    u, v = _c(u, np.int32), _c(v, np.int32)
    lab = np.empty(n, np.int32)
    c = _load().oracle_uf_cc(n, u.shape[0], _p32(u), _p32(v), _p32(lab))
    return lab, int(c)


def closure_cc(n: int, u, v):
    """Warshall closure labelling for n <= 64."""
    if n > 64:
        raise ValueError("closure oracle is for n <= 64")
    u, v = _c(u, np.int32), _c(v, np.int32)
    lab = np.empty(max(n, 1), np.int32)
    c = _load().oracle_closure_cc(n, u.shape[0], _p32(u), _p32(v), _p32(lab))
    return lab[:n].copy(), int(c)


def labels(g, method: str = "uf"):
    """Canonical labels of an ``inputs.Graph`` via the chosen oracle."""
    if method == "uf":
        return uf_cc(g.n, g.u, g.v)
    if method == "bfs":
        off, adj = csr_build(g.n, g.u, g.v, dedup=False)
        return bfs_cc(g.n, off, adj)
    if method == "closure":
        return closure_cc(g.n, g.u, g.v)
    raise ValueError(method)


# ---- batch-incremental connectivity (Appendix "ConnectIt: Streaming") ------

class Incremental:
    """Insert/IsConnected applied batch after batch in issue order."""

    def __init__(self, n: int):
        self.n = n
        self.P = np.empty(n, np.int32)
        _load().oracle_uf_init(n, _p32(self.P))

    def insert(self, u, v):
        u, v = _c(u, np.int32), _c(v, np.int32)
        _load().oracle_uf_insert(self.n, _p32(self.P), u.shape[0], _p32(u), _p32(v))

    def query(self, a, b):
        a, b = _c(a, np.int32), _c(b, np.int32)
        out = np.empty(max(a.shape[0], 1), np.uint8)
        _load().oracle_uf_query(self.n, _p32(self.P), a.shape[0], _p32(a), _p32(b), out.ctypes.data_as(_u8p))
        return out[: a.shape[0]].copy()

    def labels(self):
        lab = np.empty(self.n, np.int32)
        c = _load().oracle_uf_labels(self.n, _p32(self.P), _p32(lab))
        return lab, int(c)


# ---- spanning forest (Section 2; appendix "ConnectIt: Spanning Forest") -----

FOREST_OK, FOREST_BAD_ID, FOREST_NOT_AN_EDGE, FOREST_CYCLE, FOREST_WRONG_SPAN = 0, 1, 2, 3, 4


def forest_check(g, fu, fv) -> int:
    """0 iff the edges (fu[i], fv[i]) form a spanning forest of the graph
    ``g`` (an ``inputs.Graph``): every edge is an edge of g, none closes a
    cycle, and they connect exactly what g connects.  A spanning forest is
    not unique, so this checks the definition instead of comparing edges."""
    off, adj = csr_build(g.n, g.u, g.v, dedup=True)
    lab, _ = uf_cc(g.n, g.u, g.v)
    return forest_check_csr(g.n, off, adj, lab, fu, fv)


def forest_check_csr(n: int, offsets, adj, labels_g, fu, fv) -> int:
    """forest_check against a prepared CSR (rows sorted, deduplicated) and the
    graph's canonical labels."""
    off, adj = _c(offsets, np.int64), _c(adj, np.int32)
    lab = _c(labels_g, np.int32)
    fu, fv = _c(fu, np.int32), _c(fv, np.int32)
    z = np.zeros(1, np.int32)
    return int(_load().oracle_forest_check(n, _p64(off), _p32(adj) if adj.size else _p32(z), _p32(lab), fu.shape[0],
                                           _p32(fu) if fu.size else _p32(z), _p32(fv) if fv.size else _p32(z)))


def msf_weight(n: int, u, v, w):
    """Exact minimum spanning forest weight (Kruskal) of an undirected
    weighted pair list, and its edge count.  The reference for the
    approximate MSF of Section 5.1: a (1 + eps) approximation must weigh at
    most (1 + eps) times this."""
    u, v = _c(u, np.int32), _c(v, np.int32)
    w = _c(w, np.float64)
    k = np.zeros(1, np.int64)
    z32, z64 = np.zeros(1, np.int32), np.zeros(1, np.float64)
    total = _load().oracle_msf_weight(n, u.shape[0], _p32(u) if u.size else _p32(z32), _p32(v) if v.size else _p32(z32),
                                      (w if w.size else z64).ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _p64(k))
    return float(total), int(k[0])


def amsf_buckets(n: int, u, v, w, eps: float, max_buckets: int = 4096):
    """Bucket boundaries of the approximate MSF of Section 5.1 and the
    number of forest edges each bucket contributes.

    Boundaries: t_0 = the smallest weight, t_{i+1} = t_i * (1 + eps) in
    double, rounded down to float; an edge lies in the largest bucket i with
    t_i <= w.  Processing the buckets in order (a spanning forest per bucket
    over the earlier buckets' components) is Kruskal's algorithm on weights
    rounded down to t_i, so the per-bucket edge counts are the same for every
    forest the method can return.  Returns (thresholds float32 of nb + 1
    entries, counts int64 of nb entries).  Raises ValueError on a weight
    that is not finite and > 0 or when more than max_buckets are needed."""
    u, v = _c(u, np.int32), _c(v, np.int32)
    w = _c(w, np.float32)
    t = np.zeros(max_buckets + 1, np.float32)
    cnt = np.zeros(max(max_buckets, 1), np.int64)
    if u.size == 0:
        return t[:1][:0], cnt[:0]
    nb = _load().oracle_amsf_buckets(n, u.shape[0], _p32(u), _p32(v), w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                     float(eps), max_buckets, t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _p64(cnt))
    if nb == -2:
        raise ValueError("weights must be finite and > 0")
    if nb < 0:
        raise ValueError(f"more than {max_buckets} buckets")
    return t[: nb + 1].copy(), cnt[:nb].copy()


# ---- samplers with a deterministic partition -------------------------------

def kout_sample(n: int, offsets, adj, k: int, seed: int, mode: int = 0):
    """Partition produced by k-out sampling.

    Section 3.2 "k-out Sampling" and the appendix's sampling schemes: mode 0
    hybrid (first edge + k-1 seeded picks), 1 afforest (first k edges), 2
    pure (k seeded picks), 3 maxdeg (the largest-degree neighbour, the first
    on ties, + k-1 seeded picks); union the picked edges, fully compress.
    The result is the connected components of the picked sub-graph, in
    canonical-min form."""
    offsets, adj = _c(offsets, np.int64), _c(adj, np.int32)
    lab = np.empty(n, np.int32)
    c = _load().oracle_kout_sample_mode(n, _p64(offsets), _p32(adj) if adj.size else _p32(np.zeros(1, np.int32)),
                                        k, mode, seed, _p32(lab))
    return lab, int(c)


def bfs_sample(n: int, offsets, adj, tries: int, seed: int):
    """Partition produced by BFS sampling (Section 3.2 "Breadth-First Search
    Sampling"): the first seeded source whose component holds more than 10%
    of the vertices; that component relabelled to its minimum member."""
    offsets, adj = _c(offsets, np.int64), _c(adj, np.int32)
    lab = np.empty(n, np.int32)
    t = _load().oracle_bfs_sample(n, _p64(offsets), _p32(adj) if adj.size else _p32(np.zeros(1, np.int32)),
                                  tries, seed, _p32(lab))
    return lab, int(t)


def splitmix_out(state: int, i: int) -> int:
    """Output i of splitmix64 seeded with `state` (counter mode)."""
    return int(_load().oracle_splitmix_out(state, i))


def bfs_levels(n: int, offsets, adj, source: int, cap: int):
    """BFS from source for at most cap levels: (reached, levels expanded)."""
    offsets, adj = _c(offsets, np.int64), _c(adj, np.int32)
    lv = np.zeros(1, np.int32)
    r = _load().oracle_bfs_levels(n, _p64(offsets), _p32(adj) if adj.size else _p32(np.zeros(1, np.int32)),
                                  source, cap, _p32(lv))
    return int(r), int(lv[0])


def bfs_budget(n: int, offsets, adj, source: int, cap: int, edge_budget: int):
    """BFS that expands whole levels while the scanned adjacency entries stay
    within edge_budget and at most cap levels: (reached, levels)."""
    offsets, adj = _c(offsets, np.int64), _c(adj, np.int32)
    lv = np.zeros(1, np.int32)
    r = _load().oracle_bfs_budget(n, _p64(offsets), _p32(adj) if adj.size else _p32(np.zeros(1, np.int32)),
                                  source, cap, edge_budget, _p32(lv))
    return int(r), int(lv[0])


FEATURE_TAG = 0x66656174       # "feat": stream of the selector's draws
FEATURE_SAMPLES = 4096
PROBE_LEVELS = 4
PROBE_EDGES = 1024
PROBES = 16


def sampled_features(n: int, offsets, adj, seed: int):
    """The selector's sampled features, from their definitions (FP64):
    vertices v_i = splitmix(key, i) mod n for i < 4096 with key =
    splitmix(seed, "feat"); over the drawn vertices that have an edge, with
    f = the first entry of v's row: 9 = mean [f < v], 10 = mean
    log2(1 + |v - f|) / log2(n + 1), 11 = mean log2(1 + deg f); then
    whole-level BFSs from splitmix(key, 4096 + p) mod n, p < 16, each within
    4 levels and 1024 scanned entries: 12 = mean levels, 13 = mean reached / n."""
    off = np.asarray(offsets, np.int64)
    a = np.asarray(adj)
    key = splitmix_out(seed, FEATURE_TAG)
    cnt = down = loc = hub = 0.0
    for i in range(FEATURE_SAMPLES):
        v = splitmix_out(key, i) % n
        if off[v + 1] > off[v]:
            f = int(a[off[v]])
            cnt += 1
            down += f < v
            loc += np.log2(1.0 + abs(v - f)) / np.log2(n + 1.0)
            hub += np.log2(1.0 + float(off[f + 1] - off[f]))
    lv = rc = 0.0
    for p in range(PROBES):
        src = splitmix_out(key, FEATURE_SAMPLES + p) % n
        reached, levels = bfs_budget(n, off, a, src, PROBE_LEVELS, PROBE_EDGES)
        lv += levels
        rc += reached
    out = {9: down / cnt if cnt else 0.0, 10: loc / cnt if cnt else 0.0, 11: hub / cnt if cnt else 0.0,
           12: lv / PROBES, 13: rc / PROBES / n}
    return out


def degree_features(offsets):
    """The selector's degree features (indices 0-8, 14, 15) from the definition."""
    d = np.diff(np.asarray(offsets, np.int64)).astype(np.float64)
    n, m = d.size, d.sum()
    mean = d.mean()
    sd = d.std()
    skew = float(np.mean((d - mean) ** 3) / sd ** 3) if sd > 0 else 0.0
    return {0: np.log2(n), 1: np.log2(m + 1), 2: m / n, 3: sd / mean if mean > 0 else 0.0,
            4: d.max() / mean if mean > 0 else 0.0, 5: np.mean(d == 0), 6: np.mean(d == 1), 7: np.mean(d <= 2),
            8: skew, 14: float(m / n < 3), 15: np.log2(d.max() + 1)}


def degree_order(n: int, offsets):
    """The renumbering of the degree-ordered ingest (a layout choice, not a
    step of the paper's method): original vertex ids sorted by decreasing
    degree, ties by smaller id, where a degree above 2^b - 1 (b = the bits of
    n - 1, at least 1) counts as 2^b - 1.  Returns orig_of (position ->
    original id) and new_of (its inverse)."""
    d = np.diff(np.asarray(offsets, np.int64))
    bits = 1
    while bits < 31 and (1 << bits) < n:
        bits += 1
    d = np.minimum(d, (1 << bits) - 1)
    orig_of = np.lexsort((np.arange(n), -d)).astype(np.int32)
    new_of = np.empty(n, np.int32)
    new_of[orig_of] = np.arange(n, dtype=np.int32)
    return orig_of, new_of


def identify_frequent(labels_arr) -> int:
    """Most frequent label (Algorithm 1, IdentifyFrequent); ties go to the
    smallest label.  ``np.argmax`` returns the first maximum, i.e. the
    smallest label among those with the highest count."""
    lab = np.asarray(labels_arr)
    if lab.size == 0:
        return -1
    counts = np.bincount(lab.astype(np.int64))
    return int(np.argmax(counts))


def partial_labelling_ok(sample_labels, true_labels) -> bool:
    """Partial connectivity labelling (Section 2): equal sample labels imply
    the same true component, i.e. every sample class sits inside one
    component."""
    s = np.asarray(sample_labels, np.int64)
    t = np.asarray(true_labels, np.int64)
    first = np.full(int(s.max()) + 1 if s.size else 1, -1, np.int64)
    order = np.arange(s.shape[0])
    # record, for each sample class, the true label of its first member
    rev = order[::-1]
    first[s[rev]] = t[rev]
    return bool(np.all(first[s] == t))


# CSR preconditions (Section 2's CSR format: offsets of n + 1 entries with
# offsets[n] = m; Section 3.1's skip of the frequent component needs an
# undirected, i.e. symmetric, adjacency).  Bits: 1 offsets[0] != 0,
# 2 offsets[n] != m, 4 a row with decreasing offsets or a bound outside
# [0, m], 8 an id outside [0, n), 16 an entry (v, w) without (w, v).
CSR_OFFSET0, CSR_OFFSETN, CSR_MONOTONE, CSR_ID_RANGE, CSR_ASYMMETRIC = 1, 2, 4, 8, 16


def csr_validate(n: int, offsets, adj, check_symmetric: bool = True) -> dict:
    """Checks a CSR against those preconditions, row by row, with plain
    Python sets and counters.  Symmetry is checked only when the structure
    and ids are sound: as set membership when every row is ascending (the
    count and first row of the entries without a reverse are reported), else
    as equality of the multisets {(v, w)} and {(w, v)} (row unknown: -1)."""
    off = [int(x) for x in np.asarray(offsets).ravel()]
    a = [int(x) for x in np.asarray(adj).ravel()]
    m = len(a)
    failed, bad, first = 0, 0, None

    def flag(bit, row):
        nonlocal failed, first
        failed |= bit
        first = row if first is None else min(first, row)

    if off[0] != 0:
        flag(CSR_OFFSET0, 0)
    if off[n] != m:
        flag(CSR_OFFSETN, n - 1)
    rows_sorted = True
    good = []
    for v in range(n):
        b, e = off[v], off[v + 1]
        if b < 0 or e < b or e > m:
            flag(CSR_MONOTONE, v)
            continue
        good.append(v)
        row = a[b:e]
        for w in row:
            if w < 0 or w >= n:
                flag(CSR_ID_RANGE, v)
                bad += 1
        if any(row[i + 1] < row[i] for i in range(len(row) - 1)):
            rows_sorted = False
    checked = 0
    if check_symmetric and failed == 0:
        checked = 1 if (rows_sorted or m == 0) else 2
        if m > 0 and rows_sorted:
            rowsets = [set(a[off[v]:off[v + 1]]) for v in range(n)]
            for v in range(n):
                for w in a[off[v]:off[v + 1]]:
                    if v not in rowsets[w]:
                        flag(CSR_ASYMMETRIC, v)
                        bad += 1
        elif m > 0:
            from collections import Counter
            fwd = Counter((v, w) for v in range(n) for w in a[off[v]:off[v + 1]])
            rev = Counter((w, v) for (v, w), c in fwd.items() for _ in range(c))
            if fwd != rev:
                failed |= CSR_ASYMMETRIC
    return {"failed": failed, "rows_sorted": int(rows_sorted), "symmetry_checked": checked,
            "bad_entries": bad, "first_bad_row": -1 if (failed == 0 or first is None) else first}
