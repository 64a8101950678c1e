"""Full-size workloads, built and launched the way bench.py times them:
R-MAT 2^24 (deduplicated int32 CSR), the 256^3 bond-percolated grid, and
R-MAT 2^27 with int64 offsets.  Every sampling x finish combination must
give the canonical labels (appendix "Correctness for Sampling Algorithms"
and the finish algorithms' correctness: each combination is exact), so each
variant's labels and component count are compared element by element with
the oracle's sequential union-find over the same pair list, computed once
per graph."""
import sys

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


def _note(msg):
    print(f"[fullsize] {msg}", file=sys.stderr, flush=True)


class Loaded:
    """A workload's device CSR and the oracle's labels (host and device)."""

    def __init__(self, ctx, g, dedup=True, o64=False):
        _note(f"oracle labels for {g}")
        self.g = g
        self.want, self.wc = oracle.uf_cc(g.n, g.u, g.v)
        dev = ctx.torch_device
        self.want_dev = torch.from_numpy(self.want).to(dev)
        self.csr = b.build_csr(ctx, g.n, torch.from_numpy(g.u).to(dev), torch.from_numpy(g.v).to(dev),
                               dedup=dedup, offsets_64bit=o64)
        self.labels = torch.empty(g.n, dtype=torch.int32, device=dev)
        self.ncomp = torch.empty(1, dtype=torch.int64, device=dev)

    def check(self, ctx, variants):
        for v in variants:
            _note(f"{self.g} {v.name()} kout_mode={v.kout_mode} k={v.kout_k}")
            self.labels.fill_(-1)
            b.connectivity_csr(ctx, self.csr, v, labels=self.labels, ncomp=self.ncomp)
            torch.cuda.synchronize()
            ctx.sync_status()
            assert int(self.ncomp.item()) == self.wc, v.name()
            if not torch.equal(self.labels, self.want_dev):
                got = self.labels.cpu().numpy()
                bad = np.flatnonzero(got != self.want)
                raise AssertionError(f"{v.name()}: {len(bad)} labels differ, first at {bad[0]}: "
                                     f"{got[bad[0]]} != {self.want[bad[0]]}")


def _edge_choice_rows():
    base = b.default_variant()
    return [base.copy(kout_mode=b.KOUT_AFFOREST), base.copy(kout_mode=b.KOUT_PURE),
            base.copy(kout_k=1), base.copy(kout_k=3), base.copy(kout_mode=b.KOUT_AFFOREST, kout_k=1),
            base.copy(kout_mode=b.KOUT_MAXDEG)]


@pytest.fixture(scope="module")
def rmat24(ctx):
    L = Loaded(ctx, inputs.workload_rmat(24, 8, seed=2))
    assert L.csr.m == 263_432_958
    yield L
    del L


@pytest.fixture(scope="module")
def grid(ctx):
    yield Loaded(ctx, inputs.workload_grid3d(256, 0.35, seed=3))


def test_rmat_2_24_default(ctx, rmat24):
    rmat24.check(ctx, [b.default_variant()])


def test_rmat_2_24_every_variant(ctx, rmat24):
    """The 80 sampling x finish variants of the main table, the 76 further
    finishes under each sampler, and the k-out edge-choice rows."""
    rmat24.check(ctx, b.all_variants(extended=True) + _edge_choice_rows())


def test_rmat_2_24_degree_ordered_mapped(ctx, rmat24):
    """The degree-ordered CSR of the same pairs (as bench.py times it), every
    variant of the main table and the edge-choice rows: labels in the
    original numbering equal the oracle's."""
    dev = ctx.torch_device
    g = rmat24.g
    d = b.build_csr_degree_order(ctx, g.n, torch.from_numpy(g.u).to(dev), torch.from_numpy(g.v).to(dev))
    assert d.m == rmat24.csr.m
    for v in b.all_variants() + _edge_choice_rows():
        _note(f"{g} mapped {v.name()} kout_mode={v.kout_mode} k={v.kout_k}")
        rmat24.labels.fill_(-1)
        b.connectivity_csr_mapped(ctx, d, v, labels=rmat24.labels, ncomp=rmat24.ncomp)
        torch.cuda.synchronize()
        ctx.sync_status()
        assert int(rmat24.ncomp.item()) == rmat24.wc, v.name()
        assert torch.equal(rmat24.labels, rmat24.want_dev), v.name()
    del d


def test_grid_256_cubed_every_variant(ctx, grid):
    grid.check(ctx, [b.default_variant()] + b.all_variants(extended=True) + _edge_choice_rows())


@pytest.mark.timeout(1200)
def test_rmat_2_27_int64_offsets_main_variants(ctx):
    """R-MAT 2^27 (about 2.1e9 adjacency entries, int64 offsets): the 80
    variants of the main table."""
    L = Loaded(ctx, inputs.workload_rmat(27, 8, seed=4), o64=True)
    assert L.csr.offsets.dtype == torch.int64
    L.check(ctx, [b.default_variant()] + b.all_variants())
    del L
    torch.cuda.empty_cache()


def test_amsf_rmat_2_24(ctx, rmat24):
    """Approximate MSF (Section 5.1) on R-MAT 2^24 with exponential weights of
    mean 1, eps = 0.25: labels equal the oracle's, the forest is valid, every
    returned weight is its edge's weight, and the per-bucket forest edge
    counts equal the oracle's bucketed Kruskal (which makes the forest a
    minimum one for the rounded weights, hence within 1 + eps of the
    minimum).  The oracle works from the generator's pair list."""
    g, d = rmat24.g, rmat24.csr
    dev = ctx.torch_device
    off_d = d.offsets.cpu().numpy()
    rows_d = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(off_d))
    wt = torch.from_numpy(inputs.pair_weights(g.n, rows_d, d.adj.cpu().numpy(), seed=77)).to(dev)
    del rows_d, off_d
    keep = g.u != g.v
    pu, pv = g.u[keep], g.v[keep]
    pw = inputs.pair_weights(g.n, pu, pv, seed=77)
    _note("oracle: csr, buckets")
    want, wc = rmat24.want, rmat24.wc
    off, adj = oracle.csr_build(g.n, g.u, g.v, True)
    t, cnt = oracle.amsf_buckets(g.n, pu, pv, pw, 0.25)
    for lf in (b.amsf_options().light_fraction, 0.0):
        _note(f"amsf rmat24 light_fraction={lf}")
        lab, eu, ev, ew, ne, tw = b.amsf_csr(ctx, d, wt, b.amsf_options(epsilon=0.25, light_fraction=lf))
        torch.cuda.synchronize()
        ctx.sync_status()
        k = int(ne.item())
        fu, fv, fw = eu[:k].cpu().numpy(), ev[:k].cpu().numpy(), ew[:k].cpu().numpy()
        assert np.array_equal(lab.cpu().numpy(), want) and k == g.n - wc, lf
        assert oracle.forest_check_csr(g.n, off, adj, want, fu, fv) == oracle.FOREST_OK, lf
        assert np.array_equal(fw, inputs.pair_weights(g.n, fu, fv, seed=77)), lf
        fb = np.searchsorted(t, fw, side="right") - 1
        assert np.array_equal(np.bincount(fb, minlength=len(cnt)), cnt), lf
        assert abs(float(tw.item()) - float(np.sum(fw, dtype=np.float64))) < 1e-6 * float(tw.item())


def test_map_and_gather_edges_rmat_2_24(ctx, rmat24):
    """The calibration primitives at full size (hub rows far above a
    wave's 4096-entry limit): MapEdges gives every degree, GatherEdges the
    sum of a value over each row, as numpy computes them from the CSR."""
    d = rmat24.csr
    off = d.offsets.cpu().numpy().astype(np.int64)
    deg = np.diff(off)
    got = b.calib_edges(d).cpu().numpy()
    assert np.array_equal(got, deg.astype(np.int32))
    vals = ((np.arange(d.n, dtype=np.int64) * 7 + 3) % 1000).astype(np.int32)
    gv = b.calib_edges(d, torch.from_numpy(vals).to(ctx.torch_device)).cpu().numpy()
    adj = d.adj.cpu().numpy()
    csum = np.concatenate([[0], np.cumsum(vals[adj].astype(np.int64))])
    want = csum[off[1:]] - csum[off[:-1]]
    assert np.array_equal(gv.astype(np.int64), want)


def test_serving_trace_rmat_2_24_every_answer(ctx, rmat24):
    """The serving loop at full size (the R-MAT 2^24 pairs, shuffled, as insert
    requests of log-uniform size in [1e3, 1e7] between query requests of
    [1e3, 1e6] uniform pairs, Poisson arrivals faster than the device drains
    them, so queries overlap the inserts that arrive after them): every query
    answer equals the oracle's answer against exactly the earlier inserts."""
    g = rmat24.g
    su, sv = inputs.shuffle_pairs(g.u, g.v, 5)
    rng = np.random.default_rng(41)
    types, starts, lens, A, B = [], [], [], [], []
    pe = pos = 0
    for i in range(80):
        t = int(rng.random() < 0.5)
        if t == 0 and pe < su.size:
            k = min(inputs.log_uniform_int(1e3, 1e7, rng.random()), su.size - pe)
            A.append(su[pe:pe + k])
            B.append(sv[pe:pe + k])
            pe += k
        else:
            t = 1
            k = inputs.log_uniform_int(1e3, 1e6, rng.random())
            qa, qb = inputs.query_pairs(g.n, k, seed=4000 + i)
            A.append(qa)
            B.append(qb)
        types.append(t)
        starts.append(pos)
        lens.append(k)
        pos += k
    types, starts, lens = np.array(types, np.int32), np.array(starts, np.int64), np.array(lens, np.int64)
    A = np.concatenate(A).astype(np.int32)
    B = np.concatenate(B).astype(np.int32)
    arrivals = np.cumsum(rng.exponential(50e-6, types.size))
    srv = b.Server(ctx, g.n, budget_bytes=1 << 30, num_streams=2, max_inflight=32)
    assert srv.stamped
    _note(f"serving trace: {types.size} requests, {int(lens[types == 0].sum())} inserts, "
          f"{int(lens[types == 1].sum())} queries")
    # payloads and answers in pinned host memory, as the benchmark serves
    # them: the kernels read and answer them in place
    ta, tb = torch.from_numpy(A).pin_memory(), torch.from_numpy(B).pin_memory()
    to = torch.zeros(A.size, dtype=torch.uint8).pin_memory()
    got, lat = srv.run_trace(types, arrivals, starts, lens, ta.numpy(), tb.numpy(), to.numpy())
    inc = oracle.Incremental(g.n)
    for t, s, k in zip(types, starts, lens):
        sl = slice(s, s + k)
        if t == 0:
            inc.insert(A[sl], B[sl])
        else:
            assert np.array_equal(got[sl], inc.query(A[sl], B[sl])), (s, k)
    assert np.all(lat > 0)
    lab, nc = srv.labels()
    want, wc = inc.labels()
    assert np.array_equal(lab.cpu().numpy(), want)
    srv.close()
