"""GPU parity: the HIP path against the CPU oracle, element by element.

Inputs come from the seeded generators; expected values come only from the
oracle.  Labels are canonical minimum ids, so the bar is bit-exact."""
import numpy as np
import pytest
import torch

import oracle
from paper_2008_03909_amd import binding as b
from paper_2008_03909_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = b.Context(0)
    yield c
    c.close()


def _csr(ctx, g, dedup=True, o64=False):
    return b.build_csr(ctx, g.n, g.u, g.v, dedup=dedup, offsets_64bit=o64)


def _labels(ctx, g, variant, dedup=True, o64=False):
    d = _csr(ctx, g, dedup, o64)
    lab, nc = b.connectivity_csr(ctx, d, variant)
    torch.cuda.synchronize()
    ctx.sync_status()
    return lab.cpu().numpy(), int(nc.item())


def _suite():
    """Small graphs that span several tiles and ragged tails, plus the edge cases."""
    gs = [
        inputs.empty(1),
        inputs.empty(777),
        inputs.path(2),
        inputs.path(1000, np.arange(1000)[::-1].copy()),          # long find paths
        inputs.chain(5000, seed=3),
        inputs.star(3000, center=2999),
        inputs.clique(70),
        inputs.disjoint_union([inputs.clique(s) for s in (1, 2, 3, 5, 8, 13, 21)]),
        inputs.er(4096, 3000, seed=5),                             # many small components
        inputs.er(10_000, 80_000, seed=6),                         # giant component
        inputs.rmat(12, 8 << 12, 0.57, 0.19, 0.19, seed=7),
        inputs.grid(3, 20, 0.35, seed=8),
        inputs.grid(2, 64, 0.55, seed=9),
        inputs.relabel(inputs.grid(2, 40, 1.0, seed=1), inputs.permutation(1600, 4)),
    ]
    # a hub whose row is far longer than a block, plus isolated vertices
    hub = np.zeros(20000, np.int32)
    leaves = np.arange(1, 20001, dtype=np.int32)
    gs.append(inputs.Graph(25000, hub, leaves, "hub20000"))
    # two hubs above the grid-bin threshold joined through a path, plus a star of 5000
    h1 = np.full(40000, 7, np.int32)
    l1 = np.arange(100, 40100, dtype=np.int32)
    h2 = np.full(36000, 90000, np.int32)
    l2 = np.arange(40100, 76100, dtype=np.int32)
    gs.append(inputs.Graph(100000, np.concatenate([h1, h2, [40099]]).astype(np.int32),
                           np.concatenate([l1, l2, [40100]]).astype(np.int32), "two-heavy-hubs"))
    # twelve rows above the grid-bin threshold, several in one compaction
    # segment and in one wave, spread over eight components
    hubs = [5, 6, 7, 300, 301, 5000, 5001, 5002, 5003, 60000, 60001, 119999]
    free = np.concatenate([np.arange(10000, 60000), np.arange(60002, 119999)]).astype(np.int32)
    hu, hv, at = [], [], 0
    for i, h in enumerate(hubs):
        d = 4100 + 150 * i
        hu.append(np.full(d, h, np.int32))
        hv.append(free[at:at + d])
        at += d
    hu.append(np.array([5, 300, 60000, 7], np.int32))
    hv.append(np.array([6, 5000, 119999, 5003], np.int32))
    gs.append(inputs.Graph(120000, np.concatenate(hu), np.concatenate(hv), "twelve-heavy-rows"))
    # self-loops and duplicates
    u = np.array([0, 0, 1, 1, 2, 3, 3, 5], np.int32)
    v = np.array([0, 1, 0, 1, 2, 4, 4, 5], np.int32)
    gs.append(inputs.Graph(7, u, v, "loops+dups"))
    return gs


SUITE = _suite()


# ---- ingest -------------------------------------------------------------------------

@pytest.mark.parametrize("dedup", [True, False])
@pytest.mark.parametrize("o64", [False, True])
def test_build_csr_matches_oracle(ctx, dedup, o64):
    for g in SUITE + [inputs.workload_er_2_16()]:
        d = _csr(ctx, g, dedup, o64)
        off, adj = oracle.csr_build(g.n, g.u, g.v, dedup)
        assert d.offsets.dtype == (torch.int64 if o64 else torch.int32)
        assert np.array_equal(d.offsets.cpu().numpy().astype(np.int64), off), g
        assert np.array_equal(d.adj.cpu().numpy(), adj), g


def test_build_csr_flags_out_of_range_ids(ctx):
    g = inputs.Graph(10, np.array([1, 2, 12], np.int32), np.array([2, 3, 4], np.int32))
    d = _csr(ctx, g)
    torch.cuda.synchronize()
    with pytest.raises(b.CCError):
        ctx.sync_status()
    off, adj = oracle.csr_build(10, np.array([1, 2], np.int32), np.array([2, 3], np.int32), True)
    assert np.array_equal(d.adj.cpu().numpy(), adj)


@pytest.mark.parametrize("dedup", [True, False])
@pytest.mark.parametrize("o64", [False, True])
def test_build_csr_degree_order_matches_oracle(ctx, dedup, o64):
    """The degree-ordered ingest: the permutation equals the oracle's degree
    order of the CSR in the given numbering, and the CSR equals the oracle's
    CSR of the renumbered pairs."""
    for g in SUITE + [inputs.workload_er_2_16()]:
        d = b.build_csr_degree_order(ctx, g.n, g.u, g.v, dedup=dedup, offsets_64bit=o64)
        off0, _ = oracle.csr_build(g.n, g.u, g.v, dedup)
        orig, new = oracle.degree_order(g.n, off0)
        assert np.array_equal(d.orig_of.cpu().numpy(), orig), g
        assert np.array_equal(d.new_of.cpu().numpy(), new), g
        off, adj = oracle.csr_build(g.n, new[g.u], new[g.v], dedup)
        assert np.array_equal(d.offsets.cpu().numpy().astype(np.int64), off), g
        assert np.array_equal(d.adj.cpu().numpy(), adj), g


@pytest.mark.parametrize("vi", range(0, 156, 5))
def test_mapped_connectivity_on_the_suite(ctx, vi):
    """Labels in the original numbering from a degree-ordered CSR equal the
    oracle's labels of the original graph (every fifth variant of the 156:
    each sampler and finish family is among them)."""
    v = b.all_variants(extended=True)[vi]
    for g in SUITE:
        want, wc = oracle.labels(g)
        d = b.build_csr_degree_order(ctx, g.n, g.u, g.v)
        lab, nc = b.connectivity_csr_mapped(ctx, d, v)
        torch.cuda.synchronize()
        ctx.sync_status()
        assert int(nc.item()) == wc, (v, g)
        assert np.array_equal(lab.cpu().numpy(), want), (v, g)


def test_mapped_connectivity_with_a_random_permutation(ctx):
    """The mapped entry takes any permutation, not only the degree order."""
    for g in SUITE[8:12]:
        want, wc = oracle.labels(g)
        perm = inputs.permutation(g.n, 11).astype(np.int32)      # new id of original vertex o
        orig = np.empty(g.n, np.int32)
        orig[perm] = np.arange(g.n, dtype=np.int32)
        d0 = _csr(ctx, inputs.Graph(g.n, perm[g.u], perm[g.v]))
        dev = ctx.torch_device
        d = b.RenumberedCSR(g.n, d0.offsets, d0.adj, torch.from_numpy(orig).to(dev), torch.from_numpy(perm).to(dev))
        lab, nc = b.connectivity_csr_mapped(ctx, d)
        assert int(nc.item()) == wc and np.array_equal(lab.cpu().numpy(), want), g


def test_long_id_ordered_path(ctx):
    """A path of 2^20 vertices numbered along it: k-out links each vertex to
    its predecessor, one tree as deep as the path; every sampler and the
    compression after it still give one component labelled 0."""
    g = inputs.path(1 << 20)
    d = _csr(ctx, g)
    base = b.default_variant()
    for v in (base, base.copy(sample=b.SAMPLE_BFS), base.copy(sample=b.SAMPLE_LDD), base.copy(sample=b.SAMPLE_NONE)):
        lab, nc = b.connectivity_csr(ctx, d, v)
        torch.cuda.synchronize()
        ctx.sync_status()
        assert int(nc.item()) == 1, v.name()
        assert int(lab.max().item()) == 0 and int(lab.min().item()) == 0, v.name()

def test_csr_active_prefix(ctx):
    """The smallest x from which every row is empty, for CSRs as built and
    renumbered by degree (there it is the number of vertices with an entry:
    isolated vertices come last)."""
    for g in SUITE:
        for o64 in (False, True):
            d = _csr(ctx, g, o64=o64)
            off = d.offsets.cpu().numpy().astype(np.int64)
            want = int(np.argmax(off == off[-1]))
            assert b.csr_active_prefix(d) == want, g
            r = b.build_csr_degree_order(ctx, g.n, g.u, g.v, offsets_64bit=o64)
            roff = r.offsets.cpu().numpy().astype(np.int64)
            assert r.n_active == int(np.count_nonzero(np.diff(roff))), g
            assert r.n_active == int(np.argmax(roff == roff[-1])), g


@pytest.mark.parametrize("vi", [0, 20, 40, 60])
def test_mapped_connectivity_with_and_without_the_active_prefix(ctx, vi):
    """The call restricted to the vertices with edges and the call told
    nothing (n_active = n) give the same labels and count, both the
    oracle's."""
    v = b.all_variants()[vi]
    for g in SUITE:
        want, wc = oracle.labels(g)
        d = b.build_csr_degree_order(ctx, g.n, g.u, g.v)
        full = b.RenumberedCSR(g.n, d.offsets, d.adj, d.orig_of, d.new_of)
        for r in (d, full):
            lab, nc = b.connectivity_csr_mapped(ctx, r, v)
            torch.cuda.synchronize()
            ctx.sync_status()
            assert int(nc.item()) == wc, (v, g, r.n_active)
            assert np.array_equal(lab.cpu().numpy(), want), (v, g, r.n_active)


def test_mapped_connectivity_reports_a_broken_active_prefix(ctx):
    """n_active below the last non-empty row is reported through the
    context's error word (the parent array covers every vertex, so the call
    itself reads only valid entries)."""
    g = SUITE[8]  # many small components and isolated vertices
    d = b.build_csr_degree_order(ctx, g.n, g.u, g.v)
    assert d.n_active >= 2
    bad = b.RenumberedCSR(g.n, d.offsets, d.adj, d.orig_of, d.new_of, d.n_active - 1)
    b.connectivity_csr_mapped(ctx, bad)
    torch.cuda.synchronize()
    with pytest.raises(b.CCError):
        ctx.sync_status()
    # the context works again afterwards
    lab, nc = b.connectivity_csr_mapped(ctx, d)
    torch.cuda.synchronize()
    ctx.sync_status()
    want, wc = oracle.labels(g)
    assert int(nc.item()) == wc and np.array_equal(lab.cpu().numpy(), want)


# ---- default variant and the full variant space ----------------------------------

def test_default_variant_er_workload(ctx):
    g = inputs.workload_er_2_16()
    want, wc = oracle.labels(g)
    got, gc = _labels(ctx, g, b.default_variant(), dedup=False)
    assert gc == wc
    assert np.array_equal(got, want)


@pytest.mark.parametrize("vi", [0, 4, 9, 23, 41, 63, 79])
def test_pair_list_entry_matches_oracle(ctx, vi):
    """cc_connectivity_coo (CSR built inside the workspace) on the suite,
    including an empty pair list, self-loops and duplicates."""
    v = b.all_variants()[vi]
    for g in SUITE + [inputs.workload_er_2_16(), inputs.Graph(9, np.zeros(0, np.int32), np.zeros(0, np.int32))]:
        want, wc = oracle.labels(g)
        lab, nc = b.connectivity_coo(ctx, g.n, g.u, g.v, v)
        torch.cuda.synchronize()
        ctx.sync_status()
        assert int(nc.item()) == wc, (v, g)
        assert np.array_equal(lab.cpu().numpy(), want), (v, g)


@pytest.mark.parametrize("vi", range(156))
def test_every_variant_on_the_suite(ctx, vi):
    """The 80 main variants and the 76 with the further finishes (UF-Early,
    UF-Hooks, label propagation, non-root-based Liu-Tarjan)."""
    v = b.all_variants(extended=True)[vi]
    for g in SUITE:
        want, wc = oracle.labels(g)
        got, gc = _labels(ctx, g, v)
        assert gc == wc, (v, g)
        assert np.array_equal(got, want), (v, g)


def test_every_variant_on_all_graphs_with_six_vertices(ctx):
    g = inputs.all_graphs_on(6)
    want, wc = oracle.labels(g)
    d = _csr(ctx, g)
    for v in b.all_variants(extended=True):
        lab, nc = b.connectivity_csr(ctx, d, v)
        assert int(nc.item()) == wc, v
        assert np.array_equal(lab.cpu().numpy(), want), v


def test_rem_counterexample_graph_every_variant(ctx):
    e = np.array([[0, 2], [1, 3], [2, 5], [3, 4], [4, 5]], np.int32)
    g = inputs.Graph(6, e[:, 0], e[:, 1])
    for v in b.all_variants(extended=True):
        got, gc = _labels(ctx, g, v)
        assert gc == 1 and got.tolist() == [0] * 6, v
    bad = b.default_variant(splice=b.SPLICE_ATOMIC, find=b.FIND_COMPRESS)
    with pytest.raises(b.CCError) as ei:
        _labels(ctx, g, bad)
    assert ei.value.status == b.CC_EINVAL


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_seeds_change_nothing(ctx, seed):
    g = inputs.rmat(14, 8 << 14, 0.57, 0.19, 0.19, seed=11)
    want, _ = oracle.labels(g)
    for s in (b.SAMPLE_KOUT, b.SAMPLE_BFS, b.SAMPLE_LDD):
        v = b.default_variant(sample=s, seed=seed * 7919)
        got, _ = _labels(ctx, g, v)
        assert np.array_equal(got, want)


# ---- samplers ------------------------------------------------------------------------

@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_kout_sample_matches_oracle_partition(ctx, k, mode):
    """Every edge choice (hybrid, afforest, pure, max-degree)."""
    for g in SUITE:
        d = _csr(ctx, g)
        v = b.default_variant(kout_k=k, kout_mode=mode, seed=1234)
        lab, lmax = b.sample_csr(ctx, d, v)
        off, adj = oracle.csr_build(g.n, g.u, g.v, True)
        want, _ = oracle.kout_sample(g.n, off, adj, k, 1234, mode=mode)
        assert np.array_equal(lab.cpu().numpy(), want), g
        # IdentifyFrequent over vertices with an edge, ties to the smaller label
        deg = np.diff(off)
        if np.any(deg > 0):
            assert lmax == oracle.identify_frequent(want[deg > 0]), g


def test_bfs_sample_matches_oracle_partition(ctx):
    for g in SUITE + [inputs.disjoint_union([inputs.clique(3) for _ in range(50)])]:
        d = _csr(ctx, g)
        v = b.default_variant(sample=b.SAMPLE_BFS, seed=99)
        lab, lmax = b.sample_csr(ctx, d, v)
        off, adj = oracle.csr_build(g.n, g.u, g.v, True)
        want, t = oracle.bfs_sample(g.n, off, adj, 3, 99)
        assert np.array_equal(lab.cpu().numpy(), want), g
        st = ctx.last_stats()
        assert st["sample_success"] == t
        assert 0 <= st["sample_bottom_up"] <= st["sample_rounds"], g


def test_ldd_sample_is_a_partial_labelling_of_stars(ctx):
    bottom_up = top_down = 0
    for g in SUITE:
        d = _csr(ctx, g)
        v = b.default_variant(sample=b.SAMPLE_LDD, seed=5)
        lab, lmax = b.sample_csr(ctx, d, v)
        st = ctx.last_stats()
        assert 0 <= st["sample_bottom_up"] <= st["sample_rounds"], g
        bottom_up += st["sample_bottom_up"]
        top_down += st["sample_rounds"] - st["sample_bottom_up"]
        lab = lab.cpu().numpy()
        true, _ = oracle.labels(g)
        idx = np.arange(g.n)
        assert oracle.partial_labelling_ok(lab, true), g
        assert np.all(lab <= idx) and np.all(lab[lab] == lab), g      # stars rooted at the minimum
        # every cluster is connected inside itself: its induced sub-graph has one component
        keep = lab[g.u] == lab[g.v]
        sub, _ = oracle.uf_cc(g.n, g.u[keep], g.v[keep])
        assert np.array_equal(sub, lab), g
    # the suite runs rounds in both directions (a hub's round goes bottom-up)
    assert bottom_up > 0 and top_down > 0, (bottom_up, top_down)


# ---- incremental -----------------------------------------------------------------------

def _stream_variants():
    vs = [b.default_variant(finish=b.FIN_UF_ASYNC, find=f) for f in range(4)]
    vs += [b.default_variant(finish=b.FIN_UF_REM_CAS, splice=s, find=0) for s in range(3)]
    vs += [b.default_variant(finish=b.FIN_UF_EARLY, find=3), b.default_variant(finish=b.FIN_UF_HOOKS, find=1)]
    # type-2 streams: inserts in rounds (Shiloach-Vishkin, root-based Liu-Tarjan)
    vs += [b.default_variant(finish=b.FIN_SV)]
    vs += [b.default_variant(finish=b.FIN_LT, lt_rules=r) for r in (b.LT_CRSA, b.LT_PRSA, b.LT_PRS, b.LT_CRFA, b.LT_PRFA, b.LT_PRF)]
    return vs


@pytest.mark.parametrize("vi", range(16))
def test_incremental_matches_oracle_on_every_prefix(ctx, vi):
    v = _stream_variants()[vi]
    n = 5000
    st = b.Stream(ctx, n, v)
    inc = oracle.Incremental(n)
    rng = np.random.default_rng(vi)
    dev = ctx.torch_device
    for batch in range(12):
        k = int(rng.integers(0, 1500))
        u = rng.integers(0, n, k).astype(np.int32)
        w = rng.integers(0, n, k).astype(np.int32)
        st.insert(torch.from_numpy(u).to(dev), torch.from_numpy(w).to(dev))
        inc.insert(u, w)
        q = int(rng.integers(1, 3000))
        a = rng.integers(0, n, q).astype(np.int32)
        c = rng.integers(0, n, q).astype(np.int32)
        got = st.query(torch.from_numpy(a).to(dev), torch.from_numpy(c).to(dev)).cpu().numpy()
        assert np.array_equal(got, inc.query(a, c)), (v, batch)
    lab, nc = st.labels()
    want, wc = inc.labels()
    assert np.array_equal(lab.cpu().numpy(), want) and int(nc.item()) == wc
    st.sync_status()
    st.close()


def test_incremental_initialize_from_a_graph(ctx):
    g = inputs.er(20000, 15000, seed=3)
    d = _csr(ctx, g)
    v = b.default_variant(finish=b.FIN_UF_ASYNC)
    st = b.Stream(ctx, g.n, v)
    st.init_csr(d, v)
    inc = oracle.Incremental(g.n)
    inc.insert(g.u, g.v)
    rng = np.random.default_rng(1)
    dev = ctx.torch_device
    u = rng.integers(0, g.n, 4000).astype(np.int32)
    w = rng.integers(0, g.n, 4000).astype(np.int32)
    st.insert(torch.from_numpy(u).to(dev), torch.from_numpy(w).to(dev))
    inc.insert(u, w)
    lab, _ = st.labels()
    assert np.array_equal(lab.cpu().numpy(), inc.labels()[0])
    st.close()


def test_incremental_batch_split_and_order_invariance(ctx):
    g = inputs.rmat(13, 4 << 13, 0.57, 0.19, 0.19, seed=3)
    dev = ctx.torch_device
    want, _ = oracle.labels(g)
    for split_seed in range(3):
        st = b.Stream(ctx, g.n)
        su, sv = inputs.shuffle_pairs(g.u, g.v, split_seed)
        cuts = np.sort(np.random.default_rng(split_seed).integers(0, su.shape[0], 5))
        for part in np.split(np.arange(su.shape[0]), cuts):
            st.insert(torch.from_numpy(su[part]).to(dev), torch.from_numpy(sv[part]).to(dev))
        lab, _ = st.labels()
        assert np.array_equal(lab.cpu().numpy(), want)
        st.close()


def test_incremental_rejects_bad_ids(ctx):
    st = b.Stream(ctx, 10)
    dev = ctx.torch_device
    st.insert(torch.tensor([1, 11], dtype=torch.int32, device=dev), torch.tensor([2, 3], dtype=torch.int32, device=dev))
    torch.cuda.synchronize()
    with pytest.raises(b.CCError):
        st.sync_status()
    st.close()


# ---- calibration kernels ------------------------------------------------------------

def test_map_and_gather_edges(ctx):
    for g in SUITE + [inputs.rmat(14, 8 << 14, 0.57, 0.19, 0.19, seed=2)]:
        d = _csr(ctx, g)
        off, adj = oracle.csr_build(g.n, g.u, g.v, True)
        deg = np.diff(off).astype(np.int64)
        got = b.calib_edges(d).cpu().numpy()
        assert np.array_equal(got, deg.astype(np.int32)), g
        vals = (np.arange(g.n, dtype=np.int64) * 7 + 3) % 1000
        gv = b.calib_edges(d, torch.from_numpy(vals.astype(np.int32)).to(ctx.torch_device)).cpu().numpy()
        want = np.zeros(g.n, np.int64)
        np.add.at(want, np.repeat(np.arange(g.n), deg), vals[adj])
        assert np.array_equal(gv, want.astype(np.int32)), g


def _sym_csr(n, u, v):
    off, adj = oracle.csr_build(n, np.asarray(u, np.int32), np.asarray(v, np.int32), True)
    return np.asarray(off, np.int64), np.asarray(adj, np.int32)


def _calib_cases():
    """CSRs whose rows meet the edge-chunk boundaries in every way: a hub row
    over several chunks, a chunk spanning tens of thousands of rows (mostly
    empty), the last row the longest, no edges at all."""
    n = 10000
    yield "star", n, *_sym_csr(n, np.zeros(n - 1), np.arange(1, n))
    ids = np.arange(0, 200000, 97)
    yield "sparse path", 200000, *_sym_csr(200000, ids[:-1], ids[1:])
    yield "last hub", n, *_sym_csr(n, np.full(n - 1, n - 1), np.arange(n - 1))
    g = inputs.rmat(14, 8 << 14, 0.57, 0.19, 0.19, seed=5)
    yield "rmat", g.n + 3000, *_sym_csr(g.n + 3000, g.u, g.v)
    yield "empty", 10, np.zeros(11, np.int64), np.zeros(0, np.int32)


@pytest.mark.parametrize("o64", [False, True])
@pytest.mark.parametrize("shift", [0, 1])
def test_map_and_gather_edges_chunk_boundaries(ctx, o64, shift):
    """MapEdges / GatherEdges against their definitions on rows that cross
    the kernels' work boundaries; shift = 1 places the adjacency 4 bytes off
    16-byte alignment."""
    dev = ctx.torch_device
    for name, n, off, adj in _calib_cases():
        offs = torch.from_numpy(off.astype(np.int64 if o64 else np.int32)).to(dev)
        base = torch.zeros(adj.size + shift + 1, dtype=torch.int32, device=dev)
        base[shift:shift + adj.size] = torch.from_numpy(adj).to(dev)
        d = b.CSR(n, offs, base[shift:shift + adj.size])
        deg = np.diff(off)
        assert np.array_equal(b.calib_edges(d).cpu().numpy(), deg.astype(np.int32)), name
        vals = (np.arange(n, dtype=np.int64) * 7 + 3) % 1000
        want = np.zeros(n, np.int64)
        np.add.at(want, np.repeat(np.arange(n), deg), vals[adj])
        got = b.calib_edges(d, torch.from_numpy(vals.astype(np.int32)).to(dev)).cpu().numpy()
        assert np.array_equal(got, want.astype(np.int32)), name


def test_calib_copy(ctx):
    src = torch.randint(0, 255, (1 << 20,), dtype=torch.uint8, device=ctx.torch_device)
    dst = torch.zeros_like(src)
    b.calib_copy(src, dst)
    assert torch.equal(src, dst)
