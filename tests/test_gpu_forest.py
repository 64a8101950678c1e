"""Spanning forest (appendix "ConnectIt: Spanning Forest") against the
oracle's definition check: every returned pair is an edge, none closes a
cycle, the forest connects exactly what the graph connects and has
n - (number of components) edges; labels equal the oracle's.  A spanning
forest is not unique, so edges are checked, not compared."""
import numpy as np
import pytest
import torch

import oracle
from paper_2008_03909_amd import binding as b
from paper_2008_03909_amd import inputs

from test_gpu_parity import SUITE

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = b.Context(0)
    yield c
    c.close()


def _uf_variants():
    return [v for v in b.all_variants(extended=True) if v.finish in (b.FIN_UF_ASYNC, b.FIN_UF_EARLY, b.FIN_UF_HOOKS)
            or (v.finish == b.FIN_UF_REM_CAS and v.splice != b.SPLICE_ATOMIC)]


def _check(ctx, g, v):
    d = b.build_csr(ctx, g.n, g.u, g.v)
    lab, eu, ev, ne = b.spanning_forest_csr(ctx, d, v)
    torch.cuda.synchronize()
    ctx.sync_status()
    want, wc = oracle.labels(g)
    k = int(ne.item())
    assert np.array_equal(lab.cpu().numpy(), want), (v.name(), g)
    assert k == g.n - wc, (v.name(), g, k, g.n - wc)
    code = oracle.forest_check(g, eu[:k].cpu().numpy(), ev[:k].cpu().numpy())
    assert code == oracle.FOREST_OK, (v.name(), g, code)


@pytest.mark.parametrize("vi", range(72))
def test_forest_every_union_find_variant_on_the_suite(ctx, vi):
    v = _uf_variants()[vi]
    for g in SUITE:
        _check(ctx, g, v)


def test_forest_rmat_2_24_default_and_samplers(ctx):
    g = inputs.workload_rmat(24, 8, seed=2)
    off, adj = oracle.csr_build(g.n, g.u, g.v, True)
    want, wc = oracle.uf_cc(g.n, g.u, g.v)
    d = b.build_csr(ctx, g.n, g.u, g.v)
    base = b.default_variant()
    for v in (base, base.copy(sample=b.SAMPLE_BFS), base.copy(sample=b.SAMPLE_LDD), base.copy(sample=b.SAMPLE_NONE)):
        lab, eu, ev, ne = b.spanning_forest_csr(ctx, d, v)
        torch.cuda.synchronize()
        k = int(ne.item())
        assert np.array_equal(lab.cpu().numpy(), want) and k == g.n - wc, v.name()
        assert oracle.forest_check_csr(g.n, off, adj, want, eu[:k].cpu().numpy(), ev[:k].cpu().numpy()) == 0, v.name()


def test_forest_grid_and_failed_bfs(ctx):
    # a 3D grid with many components; BFS sampling on a graph of small
    # components fails every try, and its tree edges must not leak
    base = b.default_variant(sample=b.SAMPLE_BFS)
    _check(ctx, inputs.grid(3, 40, 0.3, seed=5), base)
    small = inputs.disjoint_union([inputs.path(50) for _ in range(30)])
    _check(ctx, small, base)


def test_forest_rejects_unsupported_finishes(ctx):
    g = inputs.er(100, 300, seed=1)
    d = b.build_csr(ctx, g.n, g.u, g.v)
    for v in (b.default_variant(finish=b.FIN_SV), b.default_variant(finish=b.FIN_LT, lt_rules=b.LT_PRF),
              b.default_variant(splice=b.SPLICE_ATOMIC), b.default_variant(finish=b.FIN_LP)):
        with pytest.raises(b.CCError) as e:
            b.spanning_forest_csr(ctx, d, v)
        assert e.value.status == b.CC_EUNSUPPORTED


def _check_mapped(ctx, g, v):
    d = b.build_csr_degree_order(ctx, g.n, g.u, g.v)
    lab, eu, ev, ne = b.spanning_forest_csr_mapped(ctx, d, v)
    torch.cuda.synchronize()
    ctx.sync_status()
    want, wc = oracle.labels(g)
    k = int(ne.item())
    assert np.array_equal(lab.cpu().numpy(), want), (v.name(), g)
    assert k == g.n - wc, (v.name(), g, k, g.n - wc)
    code = oracle.forest_check(g, eu[:k].cpu().numpy(), ev[:k].cpu().numpy())
    assert code == oracle.FOREST_OK, (v.name(), g, code)


@pytest.mark.parametrize("vi", range(0, 72, 3))
def test_forest_mapped_on_the_suite(ctx, vi):
    """The forest of the degree-ordered CSR, run on the vertices with edges
    and reported in the original numbering (every third union-find variant:
    each sampler and each finish family is among them)."""
    v = _uf_variants()[vi]
    for g in SUITE:
        _check_mapped(ctx, g, v)


def test_forest_mapped_rmat_2_24_default(ctx):
    g = inputs.workload_rmat(24, 8, seed=2)
    off, adj = oracle.csr_build(g.n, g.u, g.v, True)
    want, wc = oracle.uf_cc(g.n, g.u, g.v)
    dev = ctx.torch_device
    d = b.build_csr_degree_order(ctx, g.n, torch.from_numpy(g.u).to(dev), torch.from_numpy(g.v).to(dev))
    lab, eu, ev, ne = b.spanning_forest_csr_mapped(ctx, d, b.default_variant())
    torch.cuda.synchronize()
    ctx.sync_status()
    k = int(ne.item())
    assert np.array_equal(lab.cpu().numpy(), want) and k == g.n - wc
    assert oracle.forest_check_csr(g.n, off, adj, want, eu[:k].cpu().numpy(), ev[:k].cpu().numpy()) == 0

