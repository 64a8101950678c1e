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

