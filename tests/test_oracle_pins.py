"""Pins for the CPU oracle: closed forms, brute force, invariants, the paper's
worked example and published counts -- never the oracle against a retyped
copy of itself.  CPU only."""
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_2008_03909_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _python_components(n, edges):
    """Independent pure-Python DFS (small graphs only)."""
    nbr = [[] for _ in range(n)]
    for a, b in edges:
        nbr[a].append(b)
        nbr[b].append(a)
    lab = [-1] * n
    for s in range(n):
        if lab[s] >= 0:
            continue
        stack = [s]
        lab[s] = s
        while stack:
            x = stack.pop()
            for y in nbr[x]:
                if lab[y] < 0:
                    lab[y] = s
                    stack.append(y)
    return np.array(lab, np.int32)


def _all_three(g):
    a, ca = oracle.labels(g, "uf")
    b, cb = oracle.labels(g, "bfs")
    assert np.array_equal(a, b) and ca == cb
    return a, ca


def _invariants(g, lab, comps):
    idx = np.arange(g.n)
    assert np.all(lab <= idx)                      # canonical labels are minima
    assert np.all(lab[lab] == lab)                 # idempotent
    assert comps == int(np.sum(lab == idx))        # count = number of roots
    assert np.all(lab[g.u] == lab[g.v])            # every edge inside one class


# ---- closed forms ------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 1000])
def test_empty_graph_is_n_singletons(n):
    g = inputs.empty(n)
    lab, c = _all_three(g)
    assert c == n and np.array_equal(lab, np.arange(n))


@pytest.mark.parametrize("n", [2, 3, 50, 4097])
def test_path_any_order_is_one_component(n):
    for g in (inputs.path(n), inputs.chain(n, seed=11),
              inputs.path(n, np.arange(n)[::-1].copy())):
        lab, c = _all_three(g)
        assert c == 1 and np.all(lab == 0)
        _invariants(g, lab, c)


def test_disjoint_cliques_count_and_labels():
    sizes = [1, 2, 3, 5, 8, 13]
    g = inputs.disjoint_union([inputs.clique(s) for s in sizes])
    lab, c = _all_three(g)
    assert c == len(sizes)
    starts = np.cumsum([0] + sizes[:-1])
    expect = np.repeat(starts, sizes)
    assert np.array_equal(lab, expect)


@pytest.mark.parametrize("center", [0, 5, 99])
def test_star_and_complete_graph(center):
    g = inputs.star(100, center)
    lab, c = _all_three(g)
    assert c == 1 and np.all(lab == 0)
    g = inputs.clique(40)
    lab, c = _all_three(g)
    assert c == 1 and np.all(lab == 0)


def test_grid_percolation_extremes():
    full = inputs.grid(3, 6, 1.0, seed=3)
    assert full.num_pairs == 3 * 6 * 6 * 5
    lab, c = _all_three(full)
    assert c == 1
    none = inputs.grid(3, 6, 0.0, seed=3)
    lab, c = _all_three(none)
    assert c == 6 ** 3 and np.array_equal(lab, np.arange(216))
    full2 = inputs.grid(2, 9, 1.0, seed=1)
    assert full2.num_pairs == 2 * 9 * 8
    assert _all_three(full2)[1] == 1


def test_disjoint_union_adds_component_counts():
    parts = [inputs.er(300, 200, seed=s) for s in range(4)]
    total = sum(oracle.labels(p)[1] for p in parts)
    assert oracle.labels(inputs.disjoint_union(parts))[1] == total


# ---- worked example from the paper ---------------------------------------------

def _read_golden(name):
    d = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, *vals = line.split()
            d[k] = [int(x) for x in vals]
    return d


def test_rem_counterexample_graph_is_connected():
    d = _read_golden("rem_counterexample.txt")
    e = np.array(d["edges"], np.int32).reshape(-1, 2)
    g = inputs.Graph(d["n"][0], e[:, 0], e[:, 1])
    for method in ("uf", "bfs", "closure"):
        lab, c = oracle.labels(g, method)
        assert c == d["components"][0]
        assert lab.tolist() == d["labels"]


# ---- brute force ------------------------------------------------------------------

# Number of connected labelled graphs on k vertices, OEIS A001187.
CONNECTED_LABELLED = {1: 1, 2: 1, 3: 4, 4: 38, 5: 728, 6: 26704}


@pytest.mark.parametrize("k", [3, 4, 5, 6])
def test_all_labelled_graphs_on_k_vertices(k):
    """Every labelled graph on k vertices at once (disjoint union): the three
    oracle algorithms agree and the number of connected ones is A001187(k)."""
    g = inputs.all_graphs_on(k)
    lab, c = _all_three(g)
    _invariants(g, lab, c)
    per = lab.reshape(-1, k) - (np.arange(g.n // k) * k)[:, None]
    ncomp = (per == np.arange(k)[None, :]).sum(axis=1)
    assert int(np.sum(ncomp == 1)) == CONNECTED_LABELLED[k]
    # every sub-graph: labels equal the closure oracle on that sub-graph
    if k <= 5:
        iu, iv = np.triu_indices(k, k=1)
        for gi in range(1 << iu.shape[0]):
            sel = [(int(iu[b]), int(iv[b])) for b in range(iu.shape[0]) if gi >> b & 1]
            su = np.array([a for a, _ in sel], np.int32)
            sv = np.array([b for _, b in sel], np.int32)
            cl, _ = oracle.closure_cc(k, su, sv)
            assert np.array_equal(cl, per[gi])


def test_random_small_graphs_match_closure_and_dfs():
    rng = np.random.default_rng(5)
    for trial in range(300):
        n = int(rng.integers(1, 65))
        m = int(rng.integers(0, 2 * n + 1))
        u = rng.integers(0, n, m).astype(np.int32)
        v = rng.integers(0, n, m).astype(np.int32)
        g = inputs.Graph(n, u, v)
        lab, c = _all_three(g)
        cl, cc = oracle.closure_cc(n, u, v)
        assert np.array_equal(lab, cl) and c == cc
        assert np.array_equal(lab, _python_components(n, zip(u.tolist(), v.tolist())))


def test_er_workload_invariants():
    g = inputs.workload_er_2_16()
    lab, c = _all_three(g)
    _invariants(g, lab, c)
    # average degree 16: one giant component; isolated vertices are rare
    assert np.sum(lab == 0) > 0.99 * g.n


# ---- CSR construction -------------------------------------------------------------

@pytest.mark.parametrize("dedup", [False, True])
def test_csr_build_matches_python(dedup):
    rng = np.random.default_rng(7)
    for trial in range(50):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, 120))
        u = rng.integers(0, n, m).astype(np.int32)
        v = rng.integers(0, n, m).astype(np.int32)
        off, adj = oracle.csr_build(n, u, v, dedup)
        rows = [[] for _ in range(n)]
        for a, b in zip(u.tolist(), v.tolist()):
            if a != b:
                rows[a].append(b)
                rows[b].append(a)
        rows = [sorted(set(r)) if dedup else sorted(r) for r in rows]
        assert off[0] == 0 and off[-1] == adj.shape[0]
        for x in range(n):
            assert adj[off[x]:off[x + 1]].tolist() == rows[x]


# ---- samplers ----------------------------------------------------------------------

def test_kout_first_edge_only_closed_form():
    """k = 1 keeps only v -> (smallest neighbour of v).  That functional graph
    has only 2-cycles, so its component count is (#isolated vertices) +
    (#mutual pairs u<v with min-nbr(u)=v and min-nbr(v)=u)."""
    rng = np.random.default_rng(3)
    for trial in range(30):
        n = int(rng.integers(2, 300))
        g = inputs.er(n, int(rng.integers(0, 3 * n)), seed=trial)
        off, adj = oracle.csr_build(g.n, g.u, g.v, dedup=True)
        lab, c = oracle.kout_sample(g.n, off, adj, 1, seed=9)
        deg = np.diff(off)
        first = np.where(deg > 0, adj[np.minimum(off[:-1], max(adj.shape[0] - 1, 0))] if adj.size else -1, -1)
        iso = int(np.sum(deg == 0))
        mutual = sum(1 for x in range(n) if first[x] > x and first[first[x]] == x)
        assert c == iso + mutual


def test_kout_sample_is_partial_labelling():
    for seed in range(5):
        g = inputs.er(2000, 1500, seed=seed)   # sparse: many components
        off, adj = oracle.csr_build(g.n, g.u, g.v, dedup=True)
        true, tc = oracle.labels(g)
        for k in (1, 2, 3):
            lab, c = oracle.kout_sample(g.n, off, adj, k, seed=seed)
            assert oracle.partial_labelling_ok(lab, true)
            assert c >= tc
            assert np.all(lab <= np.arange(g.n)) and np.all(lab[lab] == lab)


def test_kout_sample_star_and_clique_collapse():
    for g in (inputs.star(500, 7), inputs.clique(30)):
        off, adj = oracle.csr_build(g.n, g.u, g.v, dedup=True)
        lab, c = oracle.kout_sample(g.n, off, adj, 2, seed=1)
        assert c == 1 and np.all(lab == 0)


def test_kout_dense_er_leaves_few_components():
    """Holm et al. (k-out theorem, cited in Section 3.2): few inter-component
    edges remain.  Loose statistical check on an average-degree-16 ER graph."""
    g = inputs.workload_er_2_16()
    off, adj = oracle.csr_build(g.n, g.u, g.v, dedup=False)
    lab, c = oracle.kout_sample(g.n, off, adj, 2, seed=1)
    L = oracle.identify_frequent(lab)
    assert np.mean(lab == L) > 0.9


def test_bfs_sample_finds_the_component_of_its_source():
    g = inputs.disjoint_union([inputs.er(600, 3000, seed=1), inputs.er(400, 2000, seed=2)])
    off, adj = oracle.csr_build(g.n, g.u, g.v, dedup=True)
    true, _ = oracle.labels(g)
    lab, t = oracle.bfs_sample(g.n, off, adj, 3, seed=4)
    assert t == 0                                   # both halves exceed 10%
    cls = lab != np.arange(g.n)
    comp = true[cls][0]
    # sampled class == one true component, labelled with its minimum
    members = np.nonzero(true == comp)[0]
    assert np.array_equal(np.nonzero(lab == members.min())[0], members)
    assert oracle.partial_labelling_ok(lab, true)


def test_bfs_sample_fails_on_tiny_components():
    g = inputs.disjoint_union([inputs.clique(3) for _ in range(50)])    # each 2% of n
    off, adj = oracle.csr_build(g.n, g.u, g.v, dedup=True)
    lab, t = oracle.bfs_sample(g.n, off, adj, 3, seed=4)
    assert t == -1 and np.array_equal(lab, np.arange(g.n))


def test_bfs_sample_threshold_is_strict():
    # component of exactly n/10 vertices never qualifies; n/10 + 1 does
    for size, ok in ((10, False), (11, True)):
        g = inputs.disjoint_union([inputs.path(size), inputs.empty(100 - size)])
        off, adj = oracle.csr_build(g.n, g.u, g.v, dedup=True)
        # every try hits either the path or an isolated vertex; try many seeds
        hit = False
        for seed in range(60):
            lab, t = oracle.bfs_sample(g.n, off, adj, 1, seed=seed)
            if t == 0:
                hit = True
                assert np.all(lab[:size] == 0)
        assert hit == ok


def test_identify_frequent_fixtures():
    assert oracle.identify_frequent(np.array([3, 3, 1, 1, 2])) == 1       # tie -> smaller
    assert oracle.identify_frequent(np.array([5])) == 5
    assert oracle.identify_frequent(np.array([0, 1, 2, 3])) == 0
    assert oracle.identify_frequent(np.array([9, 4, 9, 4, 9])) == 9


# ---- batch-incremental semantics -------------------------------------------------

def test_incremental_matches_closure_on_every_prefix():
    rng = np.random.default_rng(11)
    n = 48
    inc = oracle.Incremental(n)
    eu, ev = [], []
    prev = None
    for batch in range(20):
        k = int(rng.integers(0, 6))
        u = rng.integers(0, n, k).astype(np.int32)
        v = rng.integers(0, n, k).astype(np.int32)
        inc.insert(u, v)
        eu += u.tolist()
        ev += v.tolist()
        a = rng.integers(0, n, 100).astype(np.int32)
        b = rng.integers(0, n, 100).astype(np.int32)
        got = inc.query(a, b)
        cl, _ = oracle.closure_cc(n, np.array(eu, np.int32), np.array(ev, np.int32))
        assert np.array_equal(got, (cl[a] == cl[b]).astype(np.uint8))
        lab, _ = inc.labels()
        assert np.array_equal(lab, cl)
        if prev is not None:       # answers are monotone: once connected, always
            assert np.all(cl[prev[0]] == cl[prev[1]])
        prev = (a[got == 1], b[got == 1])


# ---- selector features from their definitions -----------------------------------

def test_bfs_budget_on_a_path_closed_form():
    """Path 0-1-...-(n-1) from 0: expanding k levels scans 1 + 2(k-1)
    entries (the source has one neighbour, inner vertices two), so a budget
    of 6 allows 3 levels and 4 vertices; without limits the search expands
    eccentricity + 1 = n levels."""
    g = inputs.path(50)
    off, adj = oracle.csr_build(g.n, g.u, g.v)
    assert oracle.bfs_budget(50, off, adj, 0, 8, 6) == (4, 3)
    assert oracle.bfs_budget(50, off, adj, 0, 8, 10**9) == (9, 8)
    assert oracle.bfs_budget(50, off, adj, 0, 1000, 10**9) == (50, 50)
    assert oracle.bfs_budget(50, off, adj, 25, 3, 10**9) == (7, 3)


def test_bfs_budget_star_and_isolated():
    g = inputs.star(101, 0)           # centre 0, leaves 1..100
    off, adj = oracle.csr_build(g.n, g.u, g.v)
    assert oracle.bfs_budget(101, off, adj, 7, 8, 50) == (2, 1)     # the centre's row exceeds the budget
    # centre row fits: leaf -> centre -> all leaves -> leaves scan back (nothing new)
    assert oracle.bfs_budget(101, off, adj, 7, 8, 1 + 100 + 99) == (101, 3)
    e = inputs.empty(5)
    off, adj = oracle.csr_build(e.n, e.u, e.v)
    assert oracle.bfs_budget(5, off, adj, 3, 8, 4096) == (1, 1)


def test_bfs_budget_without_limits_agrees_with_plain_bfs():
    """Two separate searches: with no budget and a large cap, reached is the
    size of the source's component and levels its eccentricity + 1."""
    for seed in range(5):
        g = inputs.er(400, 300 + 60 * seed, seed=seed)
        off, adj = oracle.csr_build(g.n, g.u, g.v)
        lab, _ = oracle.bfs_cc(g.n, off, adj)
        for src in (0, 17, 399):
            r, lv = oracle.bfs_budget(g.n, off, adj, src, 10**6, 10**12)
            r2, lv2 = oracle.bfs_levels(g.n, off, adj, src, 0)
            assert r == int(np.sum(lab == lab[src])) == r2
            assert lv == lv2


def test_sampled_features_closed_forms():
    # path: every first neighbour is at distance 1 -> locality 1/log2(n+1);
    # the first neighbour is smaller for every v but 0
    n = 5000
    g = inputs.path(n)
    off, adj = oracle.csr_build(g.n, g.u, g.v)
    f = oracle.sampled_features(n, off, adj, 0x5eed)
    assert abs(f[10] - 1.0 / np.log2(n + 1)) < 1e-12
    key = oracle.splitmix_out(0x5eed, oracle.FEATURE_TAG)
    zeros = sum(oracle.splitmix_out(key, i) % n == 0 for i in range(oracle.FEATURE_SAMPLES))
    assert abs(f[9] - (1 - zeros / oracle.FEATURE_SAMPLES)) < 1e-12
    # complete graph: every first neighbour has degree n-1
    k = inputs.clique(40)
    off, adj = oracle.csr_build(k.n, k.u, k.v)
    f = oracle.sampled_features(40, off, adj, 3)
    assert abs(f[11] - np.log2(40)) < 1e-12
    assert f[12] == 1 and f[13] == 1.0          # one level reaches everything; 39 + 39*39 > 1024 stops the next
    # no edges: the sampled means are 0, the probe expands its isolated source
    e = inputs.empty(100)
    off, adj = oracle.csr_build(e.n, e.u, e.v)
    f = oracle.sampled_features(100, off, adj, 1)
    assert (f[9], f[10], f[11], f[12], f[13]) == (0.0, 0.0, 0.0, 1.0, 0.01)


# ---- spanning forest checker: planted mistakes must be caught --------------------

def test_forest_check_accepts_trees_and_rejects_planted_mistakes():
    g = inputs.disjoint_union([inputs.path(6), inputs.clique(4), inputs.empty(3)])   # 13 vertices, 5 components
    # a valid forest: the path's 5 edges and a star inside the clique
    fu = np.array([0, 1, 2, 3, 4, 6, 6, 6], np.int32)
    fv = np.array([1, 2, 3, 4, 5, 7, 8, 9], np.int32)
    assert oracle.forest_check(g, fu, fv) == oracle.FOREST_OK
    assert oracle.forest_check(g, fv, fu) == oracle.FOREST_OK            # orientation does not matter
    # dropping an edge leaves the path split
    assert oracle.forest_check(g, fu[1:], fv[1:]) == oracle.FOREST_WRONG_SPAN
    # an extra clique edge closes a cycle
    assert oracle.forest_check(g, np.append(fu, 7), np.append(fv, 8)) == oracle.FOREST_CYCLE
    # a pair that is not an edge (0 and 2 are not adjacent on the path)
    bad_u = fu.copy(); bad_u[1] = 0
    assert oracle.forest_check(g, bad_u, fv) == oracle.FOREST_NOT_AN_EDGE
    # an id outside [0, n)
    assert oracle.forest_check(g, np.append(fu, 13), np.append(fv, 0)) == oracle.FOREST_BAD_ID
    # the empty graph's forest is empty
    e = inputs.empty(5)
    assert oracle.forest_check(e, np.zeros(0, np.int32), np.zeros(0, np.int32)) == oracle.FOREST_OK


def test_forest_check_on_random_graphs_against_bfs_trees():
    """BFS parent edges (computed here in plain Python) form a spanning forest;
    swapping one tree edge for a non-tree edge of the same component keeps it
    one, while duplicating a tree edge does not."""
    import collections
    for seed in range(4):
        g = inputs.er(300, 350 + 50 * seed, seed=seed)
        off, adj = oracle.csr_build(g.n, g.u, g.v)
        seen = np.zeros(g.n, bool)
        fu, fv = [], []
        for s in range(g.n):
            if seen[s]:
                continue
            seen[s] = True
            dq = collections.deque([s])
            while dq:
                x = dq.popleft()
                for y in adj[off[x]:off[x + 1]]:
                    if not seen[y]:
                        seen[y] = True
                        fu.append(x)
                        fv.append(int(y))
                        dq.append(y)
        fu, fv = np.array(fu, np.int32), np.array(fv, np.int32)
        _, c = oracle.labels(g)
        assert fu.size == g.n - c
        assert oracle.forest_check(g, fu, fv) == oracle.FOREST_OK
        assert oracle.forest_check(g, np.append(fu, fu[0]), np.append(fv, fv[0])) == oracle.FOREST_CYCLE


# ---- exact MSF weight (Kruskal) ------------------------------------------------

def test_msf_weight_closed_forms():
    # a tree is its own MSF; a cycle drops its heaviest edge; unit weights give n - c
    rng = np.random.default_rng(3)
    g = inputs.path(40)
    w = rng.uniform(0.5, 2.0, g.num_pairs)
    assert abs(oracle.msf_weight(g.n, g.u, g.v, w)[0] - w.sum()) < 1e-9
    n = 30
    cu = np.arange(n, dtype=np.int32)
    cv = ((cu + 1) % n).astype(np.int32)
    cw = rng.uniform(1, 5, n)
    tot, k = oracle.msf_weight(n, cu, cv, cw)
    assert k == n - 1 and abs(tot - (cw.sum() - cw.max())) < 1e-9
    e = inputs.er(500, 700, seed=9)
    _, c = oracle.labels(e)
    tot, k = oracle.msf_weight(e.n, e.u, e.v, np.ones(e.num_pairs))
    assert k == e.n - c and tot == e.n - c


def test_msf_weight_against_brute_force():
    """Minimum over every spanning tree of small complete graphs."""
    rng = np.random.default_rng(5)
    for n in (3, 4, 5, 6):
        pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
        for _ in range(3):
            w = rng.exponential(1.0, len(pairs))
            best = np.inf
            for sub in itertools.combinations(range(len(pairs)), n - 1):
                P = list(range(n))

                def f(x):
                    while P[x] != x:
                        x = P[x]
                    return x
                ok = True
                for i in sub:
                    ra, rb = f(pairs[i][0]), f(pairs[i][1])
                    if ra == rb:
                        ok = False
                        break
                    P[max(ra, rb)] = min(ra, rb)
                if ok:
                    best = min(best, sum(w[i] for i in sub))
            u = np.array([p[0] for p in pairs], np.int32)
            v = np.array([p[1] for p in pairs], np.int32)
            assert abs(oracle.msf_weight(n, u, v, w)[0] - best) < 1e-9


# ---- approximate MSF buckets (Section 5.1) -----------------------------------

def _spanning_forests(n, pairs):
    """Every spanning forest of a small multigraph, as index tuples."""
    P = list(range(n))

    def f(x):
        while P[x] != x:
            x = P[x]
        return x
    comps = n
    for a, b in pairs:
        ra, rb = f(a), f(b)
        if ra != rb:
            P[max(ra, rb)] = min(ra, rb)
            comps -= 1
    k = n - comps
    out = []
    for sub in itertools.combinations(range(len(pairs)), k):
        P = list(range(n))
        ok = True
        for i in sub:
            ra, rb = f(pairs[i][0]), f(pairs[i][1])
            if ra == rb:
                ok = False
                break
            P[max(ra, rb)] = min(ra, rb)
        if ok:
            out.append(sub)
    return out


def test_amsf_thresholds_closed_forms():
    """Boundaries t_0 = W_min, t_{i+1} = t_i (1 + eps) rounded down to
    float: exact for eps = 0.25 from 1.0, and one float below 1.1 for
    eps = 0.1 (round-to-nearest would give 1.1f itself)."""
    u = np.array([0, 1, 2, 3], np.int32)
    v = np.array([1, 2, 3, 4], np.int32)
    w = np.array([1.0, 1.25, 1.5625, 2.0], np.float32)
    t, cnt = oracle.amsf_buckets(5, u, v, w, 0.25)
    assert t.tolist() == [1.0, 1.25, 1.5625, 1.953125, 2.44140625]
    assert cnt.tolist() == [1, 1, 1, 1]  # a path: every edge is a forest edge
    below = np.nextafter(np.float32(1.1), np.float32(0))
    w = np.array([1.0, below, np.float32(1.1), np.nextafter(below, np.float32(0))], np.float32)
    t, cnt = oracle.amsf_buckets(5, u, v, w, 0.1)
    assert t[1] == below
    assert cnt.tolist() == [2, 2]  # 1.0 and the float under t_1 in bucket 0; t_1 and 1.1f in bucket 1
    # every weight equal: one bucket holding n - c forest edges
    t, cnt = oracle.amsf_buckets(6, np.array([0, 1, 0, 3], np.int32), np.array([1, 2, 2, 4], np.int32),
                                 np.full(4, 3.0, np.float32), 0.25)
    assert len(t) == 2 and cnt.tolist() == [3]
    # a ratio under 1 + eps: one bucket
    t, cnt = oracle.amsf_buckets(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                                 np.array([1.0, 1.2], np.float32), 0.25)
    assert cnt.tolist() == [2]
    with pytest.raises(ValueError):
        oracle.amsf_buckets(3, np.array([0], np.int32), np.array([1], np.int32), np.array([0.0], np.float32), 0.25)
    with pytest.raises(ValueError):
        oracle.amsf_buckets(3, np.array([0, 1], np.int32), np.array([1, 2], np.int32),
                            np.array([1.0, 1e30], np.float32), 0.25, max_buckets=16)


def test_amsf_counts_against_brute_force():
    """On small multigraphs, every spanning forest of minimum rounded weight
    (each weight rounded down to its bucket's boundary) has exactly the
    oracle's per-bucket counts, and the bucketed forests weigh at most
    (1 + eps) times the exact minimum."""
    rng = np.random.default_rng(11)
    for trial in range(30):
        n = int(rng.integers(3, 7))
        k = int(rng.integers(n - 1, n + 4))
        pairs = [tuple(int(x) for x in rng.choice(n, 2, replace=False)) for _ in range(k)]
        eps = float(rng.choice([0.1, 0.25, 1.0]))
        w = rng.exponential(1.0, k).astype(np.float32)
        u = np.array([p[0] for p in pairs], np.int32)
        v = np.array([p[1] for p in pairs], np.int32)
        t, cnt = oracle.amsf_buckets(n, u, v, w, eps)
        b = np.searchsorted(t, w, side="right") - 1
        rounded = t[b].astype(np.float64)
        forests = _spanning_forests(n, pairs)
        best = min(sum(rounded[i] for i in f) for f in forests)
        exact, _ = oracle.msf_weight(n, u, v, w.astype(np.float64))
        for f in forests:
            if sum(rounded[i] for i in f) <= best * (1 + 1e-12):
                assert np.bincount(b[list(f)], minlength=len(cnt)).tolist() == cnt.tolist(), trial
                assert sum(float(w[i]) for i in f) <= (1 + eps) * exact * (1 + 1e-9), trial


# ---- k-out edge choices (appendix "Sampling Schemes") -------------------------

def _csr_from_rows(rows):
    off = np.zeros(len(rows) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    adj = np.array([x for r in rows for x in r], np.int32)
    return off, adj


def test_kout_maxdeg_closed_form():
    """Two hubs (2, 3) with two leaves each, joined through the path 2-0-1-3.
    With k = 1, max-degree picks send 0 to hub 2 and 1 to hub 3 and the edge
    0-1 is never picked: two components.  The first-edge (hybrid) rule picks
    0-1 and joins everything; afforest k = 1 is hybrid k = 1."""
    rows = [[1, 2], [0, 3], [0, 4, 5], [1, 6, 7], [2], [2], [3], [3]]
    off, adj = _csr_from_rows(rows)
    lab, c = oracle.kout_sample(8, off, adj, 1, seed=3, mode=3)
    assert c == 2 and lab.tolist() == [0, 1, 0, 1, 0, 0, 1, 1]
    for mode in (0, 1):
        lab, c = oracle.kout_sample(8, off, adj, 1, seed=3, mode=mode)
        assert c == 1 and np.all(lab == 0)


def test_kout_maxdeg_ties_take_the_first():
    """Vertex 0's neighbours 1 and 2 both have degree 2; 1 and 2 each lead to
    a hub of degree 3 with two leaves.  With k = 1, 0 picks 1 (the first of
    the tie), so the components are {0, 1, 3, 5, 6} and {2, 4, 7, 8};
    taking the last of a tie would give {1, 3, 5, 6} and {0, 2, 4, 7, 8}."""
    rows = [[1, 2], [0, 3], [0, 4], [1, 5, 6], [2, 7, 8], [3], [3], [4], [4]]
    off, adj = _csr_from_rows(rows)
    lab, c = oracle.kout_sample(9, off, adj, 1, seed=3, mode=3)
    assert c == 2 and lab.tolist() == [0, 0, 2, 0, 2, 0, 0, 2, 2]


def test_kout_pure_and_afforest_are_partial_labellings():
    for seed in range(3):
        g = inputs.er(3000, 2500, seed=seed)
        off, adj = oracle.csr_build(g.n, g.u, g.v, dedup=True)
        true, tc = oracle.labels(g)
        for mode in (1, 2, 3):
            for k in (1, 2):
                lab, c = oracle.kout_sample(g.n, off, adj, k, seed=seed, mode=mode)
                assert oracle.partial_labelling_ok(lab, true) and c >= tc
        # afforest with k >= every degree picks every edge: the exact labelling
        lab, c = oracle.kout_sample(g.n, off, adj, int(np.diff(off).max()) + 1, seed=seed, mode=1)
        assert np.array_equal(lab, true)


# ---- selector degree features: closed forms of the population moments ----------

def _offsets(degrees):
    return np.concatenate([[0], np.cumsum(np.asarray(degrees, np.int64))])


def test_degree_features_star_closed_form():
    # star with 4 leaves: degrees (4,1,1,1,1), mean 8/5, variance 4 - 64/25 = 36/25,
    # sd 6/5, third central moment (2.4^3 - 4*0.6^3)/5 = 2.592 = 1.5 * sd^3
    f = oracle.degree_features(_offsets([4, 1, 1, 1, 1]))
    exp = {0: np.log2(5), 1: np.log2(9), 2: 8 / 5, 3: 0.75, 4: 2.5, 5: 0.0, 6: 0.8, 7: 0.8,
           8: 1.5, 14: 1.0, 15: np.log2(5)}
    for i, e in exp.items():
        assert abs(f[i] - e) < 1e-12, (i, f[i], e)


def test_degree_features_path_closed_form():
    # path on 4 vertices: degrees (1,2,2,1), mean 3/2, sd 1/2, symmetric -> skew 0
    f = oracle.degree_features(_offsets([1, 2, 2, 1]))
    exp = {0: 2.0, 1: np.log2(7), 2: 1.5, 3: 1 / 3, 4: 4 / 3, 5: 0.0, 6: 0.5, 7: 1.0,
           8: 0.0, 14: 1.0, 15: np.log2(3)}
    for i, e in exp.items():
        assert abs(f[i] - e) < 1e-12, (i, f[i], e)


def test_degree_features_regular_and_empty_branches():
    # K_5: every degree 4 -> sd = 0 (CV and skew take their zero branch), m/n = 4 >= 3
    f = oracle.degree_features(_offsets([4] * 5))
    exp = {0: np.log2(5), 1: np.log2(21), 2: 4.0, 3: 0.0, 4: 1.0, 5: 0.0, 6: 0.0, 7: 0.0,
           8: 0.0, 14: 0.0, 15: np.log2(5)}
    for i, e in exp.items():
        assert abs(f[i] - e) < 1e-12, (i, f[i], e)
    # K_4: m/n = 3 exactly, and the flag is strict (m/n < 3)
    assert oracle.degree_features(_offsets([3] * 4))[14] == 0.0
    # no edges: mean 0 -> CV and max/mean take their zero branch; every degree is 0 (<= 2)
    f = oracle.degree_features(_offsets([0] * 6))
    exp = {0: np.log2(6), 1: 0.0, 2: 0.0, 3: 0.0, 4: 0.0, 5: 1.0, 6: 0.0, 7: 1.0,
           8: 0.0, 14: 1.0, 15: 0.0}
    for i, e in exp.items():
        assert abs(f[i] - e) < 1e-12, (i, f[i], e)


def test_degree_features_skew_sign_and_library_moments():
    # one hub among many degree-2 vertices: right-skewed; a single low vertex
    # among many degree-5 ones: left-skewed; magnitudes against scipy's
    # population (biased) moments, an independent implementation
    from scipy import stats
    for degs, sign in (([9, 2, 2, 2, 2, 2, 3], 1), ([0, 5, 5, 5, 5, 4], -1)):
        f = oracle.degree_features(_offsets(degs))
        d = np.asarray(degs, np.float64)
        assert np.sign(f[8]) == sign
        assert abs(f[8] - stats.skew(d, bias=True)) < 1e-12
        assert abs(f[3] - stats.variation(d)) < 1e-12
        # fractions by counting
        assert f[5] == sum(x == 0 for x in degs) / len(degs)
        assert f[6] == sum(x == 1 for x in degs) / len(degs)
        assert f[7] == sum(x <= 2 for x in degs) / len(degs)
        assert f[14] == float(sum(degs) < 3 * len(degs))


# ---- partial labelling checker: planted violations must be caught ----------------

def _partial_by_pairs(s, t):
    """Definition by brute force over all pairs: s[i] == s[j] implies t[i] == t[j]."""
    k = len(s)
    return all(t[i] == t[j] for i in range(k) for j in range(k) if s[i] == s[j])


def test_partial_labelling_accepts_refinements():
    true = np.array([0, 0, 0, 3, 3, 5])
    assert oracle.partial_labelling_ok(true, true)                       # the labelling itself
    assert oracle.partial_labelling_ok(np.arange(6), true)               # identity (nothing sampled)
    assert oracle.partial_labelling_ok(np.array([0, 1, 0, 3, 4, 5]), true)
    assert oracle.partial_labelling_ok(np.array([], np.int64), np.array([], np.int64))


def test_partial_labelling_rejects_planted_violations():
    true = np.array([0, 0, 2, 2, 4])
    # a sample class spanning two true components, with the stray member first,
    # in the middle and last in the class
    for s in ([0, 0, 0, 2, 4], [2, 0, 2, 2, 4], [0, 2, 2, 2, 4], [0, 0, 2, 2, 0]):
        assert not oracle.partial_labelling_ok(np.array(s), true), s
    # one class merges everything
    assert not oracle.partial_labelling_ok(np.zeros(5, np.int64), true)
    # one violating vertex among many correct ones
    t = np.repeat(np.arange(50) * 10, 10)
    s = t.copy()
    s[257] = s[100]
    assert not oracle.partial_labelling_ok(s, t)


def test_partial_labelling_against_pairwise_brute_force():
    rng = np.random.default_rng(7)
    for _ in range(400):
        k = int(rng.integers(1, 9))
        t = rng.integers(0, 3, k)
        s = rng.integers(0, 4, k)
        assert oracle.partial_labelling_ok(s, t) == _partial_by_pairs(s, t), (s, t)


# ---- CSR preconditions -------------------------------------------------------
# Section 2 fixes the CSR format (offsets[n] = m) and Section 3.1's skip
# needs a symmetric adjacency.  Each case plants one defect (or none) and
# records which check it breaks; the oracle's checker must report exactly
# that, so a checker that accepts everything, or flags the wrong row, fails.

def test_csr_validate_reports_each_planted_defect():
    import csr_cases
    for c in csr_cases.cases():
        r = oracle.csr_validate(c.n, c.off, c.adj, c.sym)
        assert r["failed"] == c.bits, c
        if c.first is not None:
            assert r["first_bad_row"] == c.first, c
        if c.bits == 0:
            assert r["first_bad_row"] == -1 and r["bad_entries"] == 0, c
        if c.bad is not None:
            assert r["bad_entries"] == c.bad, c
        if c.sorted_rows is not None:
            assert r["rows_sorted"] == c.sorted_rows, c


def test_csr_validate_symmetry_mode_and_pairwise_definition():
    """Exact symmetry agrees with the plain pairwise definition (each entry's
    reverse is somewhere in the other row) on random small adjacency lists;
    the multiset mode runs only for unsorted rows."""
    rng = np.random.default_rng(5)
    for trial in range(60):
        n = int(rng.integers(1, 9))
        rows = [sorted(set(rng.integers(0, n, size=int(rng.integers(0, 4))).tolist())) for _ in range(n)]
        if trial % 2 == 0:          # make it symmetric
            for v in range(n):
                for w in list(rows[v]):
                    if v not in rows[w]:
                        rows[w] = sorted(rows[w] + [v])
        off = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
        adj = np.array([w for r in rows for w in r], np.int32)
        want = all(v in rows[w] for v in range(n) for w in rows[v])
        r = oracle.csr_validate(n, off, adj)
        assert (r["failed"] == 0) == want, (rows, r)
        assert r["symmetry_checked"] == 1
        rev = adj.copy()
        for v in range(n):
            rev[off[v]:off[v + 1]] = adj[off[v]:off[v + 1]][::-1]
        r2 = oracle.csr_validate(n, off, rev)
        assert (r2["failed"] == 0) == want
        if any(len(x) > 1 for x in rows):
            assert r2["symmetry_checked"] == 2 and r2["rows_sorted"] == 0


# ---- degree-ordered ingest (layout) -------------------------------------------

def test_degree_order_hand_cases():
    """Star: the centre first, then the leaves by id; path 0-1-2-3-4: the
    interior vertices (degree 2) by id, then the ends; isolated vertices
    last; equal degrees keep id order."""
    off, _ = oracle.csr_build(6, np.array([3, 3, 3, 3, 3], np.int32), np.array([0, 1, 2, 4, 5], np.int32))
    orig, new = oracle.degree_order(6, off)
    assert orig.tolist() == [3, 0, 1, 2, 4, 5]
    assert new.tolist() == [1, 2, 3, 0, 4, 5]
    off, _ = oracle.csr_build(7, np.array([0, 1, 2, 3], np.int32), np.array([1, 2, 3, 4], np.int32))
    orig, new = oracle.degree_order(7, off)
    assert orig.tolist() == [1, 2, 3, 0, 4, 5, 6]
    assert np.array_equal(new[orig], np.arange(7))


def test_degree_order_is_a_sort_by_degree_then_id():
    """On random graphs: a permutation, degrees non-increasing along it,
    ids increasing within a degree; brute-force comparison with Python's
    sorted on the (-degree, id) key."""
    rng = np.random.default_rng(3)
    for n in (1, 2, 17, 300):
        k = int(rng.integers(0, 4 * n + 1))
        u = rng.integers(0, n, k).astype(np.int32)
        v = rng.integers(0, n, k).astype(np.int32)
        off, _ = oracle.csr_build(n, u, v)
        deg = np.diff(np.asarray(off, np.int64))
        orig, new = oracle.degree_order(n, off)
        assert sorted(orig.tolist()) == list(range(n))
        assert orig.tolist() == sorted(range(n), key=lambda x: (-int(deg[x]), x))
        assert np.array_equal(new[orig], np.arange(n))


def test_degree_order_caps_degrees_at_the_id_width():
    """Without deduplication a degree can exceed n - 1; it counts as 2^b - 1
    (b = bits of n - 1), so two such vertices tie and keep id order."""
    n = 4   # b = 2, cap 3
    u = np.array([1, 1, 1, 1, 1, 2, 2, 2, 2], np.int32)
    v = np.array([0, 0, 0, 0, 3, 0, 0, 0, 3], np.int32)
    off, _ = oracle.csr_build(n, u, v, False)
    deg = np.diff(np.asarray(off, np.int64))
    assert deg.tolist() == [7, 5, 4, 2]
    orig, _ = oracle.degree_order(n, off)
    assert orig.tolist() == [0, 1, 2, 3]   # 7, 5 and 4 all count as 3
