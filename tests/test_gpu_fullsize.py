"""Full-size workloads, built and launched the way bench.py times them:
R-MAT 2^24 (deduplicated int32 CSR), the 256^3 bond-percolated grid, and
R-MAT 2^27 with int64 offsets.  Labels and component counts are compared
element by element with the oracle's sequential union-find over the same
pair list."""
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


def _check(ctx, g, variants, dedup=True, o64=False):
    want, wc = oracle.uf_cc(g.n, g.u, g.v)
    dev = ctx.torch_device
    d = b.build_csr(ctx, g.n, torch.from_numpy(g.u).to(dev), torch.from_numpy(g.v).to(dev), dedup=dedup,
                    offsets_64bit=o64)
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    ncomp = torch.empty(1, dtype=torch.int64, device=dev)
    for v in variants:
        _note(f"{g} {v.name()}")
        b.connectivity_csr(ctx, d, v, labels=labels, ncomp=ncomp)
        torch.cuda.synchronize()
        ctx.sync_status()
        assert int(ncomp.item()) == wc, v.name()
        assert np.array_equal(labels.cpu().numpy(), want), v.name()
    return d


def _spread():
    vs = b.all_variants()
    return [b.default_variant()] + [vs[i] for i in (0, 13, 24, 39, 44, 58, 66, 79)]


def test_rmat_2_24(ctx):
    g = inputs.workload_rmat(24, 8, seed=2)
    d = _check(ctx, g, _spread())
    assert d.m == 263_432_958


def test_rmat_2_24_further_finishes(ctx):
    """UF-Early, UF-Hooks, label propagation and non-root-based Liu-Tarjan
    (with k-out and without sampling) and k-out's max-degree edge choice."""
    g = inputs.workload_rmat(24, 8, seed=2)
    base = b.default_variant()
    _check(ctx, g, [base.copy(finish=b.FIN_UF_EARLY, find=b.FIND_NAIVE),
                    base.copy(finish=b.FIN_UF_HOOKS, find=b.FIND_ATOMIC_SPLIT),
                    base.copy(finish=b.FIN_LP), base.copy(sample=b.SAMPLE_NONE, finish=b.FIN_LP),
                    base.copy(sample=b.SAMPLE_NONE, finish=b.FIN_UF_EARLY, find=b.FIND_COMPRESS),
                    base.copy(kout_mode=b.KOUT_MAXDEG),
                    base.copy(finish=b.FIN_LT, lt_rules=b.LT_NONROOT["CUSA"]),
                    base.copy(finish=b.FIN_LT, lt_rules=b.LT_NONROOT["EUF"]),
                    base.copy(sample=b.SAMPLE_NONE, finish=b.FIN_LT, lt_rules=b.LT_NONROOT["PUSA"])])


def test_grid_256_cubed(ctx):
    g = inputs.workload_grid3d(256, 0.35, seed=3)
    _check(ctx, g, _spread())


@pytest.mark.slow
def test_rmat_2_27_int64_offsets(ctx):
    g = inputs.workload_rmat(27, 8, seed=4)
    vs = b.all_variants()
    d = _check(ctx, g, [b.default_variant(), vs[44], vs[79]], o64=True)
    assert d.offsets.dtype == torch.int64


def test_amsf_rmat_2_24(ctx):
    """Approximate MSF (Section 5.1) on R-MAT 2^24 with exponential weights of
    mean 1, eps = 0.25: labels equal the oracle's, the forest is valid, every
    returned weight is its edge's weight, and the per-bucket forest edge
    counts equal the oracle's bucketed Kruskal (which makes the forest a
    minimum one for the rounded weights, hence within 1 + eps of the
    minimum).  The oracle works from the generator's pair list."""
    g = inputs.workload_rmat(24, 8, seed=2)
    dev = ctx.torch_device
    d = b.build_csr(ctx, g.n, torch.from_numpy(g.u).to(dev), torch.from_numpy(g.v).to(dev))
    off_d = d.offsets.cpu().numpy()
    rows_d = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(off_d))
    wt = torch.from_numpy(inputs.pair_weights(g.n, rows_d, d.adj.cpu().numpy(), seed=77)).to(dev)
    del rows_d, off_d
    keep = g.u != g.v
    pu, pv = g.u[keep], g.v[keep]
    pw = inputs.pair_weights(g.n, pu, pv, seed=77)
    _note("oracle: labels, csr, buckets")
    want, wc = oracle.uf_cc(g.n, g.u, g.v)
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
