"""The no-allocation entry point (cc_connectivity_csr_noalloc) against the
allocating one (cc_connectivity_csr) through the C ABI: two calls in a row
per variant, the second on a smaller graph (the shared scratch array keeps
the first call's contents), labels and counts equal element by element to
the allocating call's and to the oracle's; sizes beyond the array are
refused with CC_ENOMEM."""
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


def _variants():
    v = b.default_variant()
    return [v, v.copy(sample=b.SAMPLE_BFS, finish=b.FIN_SV), v.copy(sample=b.SAMPLE_LDD, finish=b.FIN_LT,
                                                                    lt_rules=b.LT_PRF),
            v.copy(sample=b.SAMPLE_NONE, finish=b.FIN_UF_ASYNC, find=b.FIND_ATOMIC_HALVE)]


def test_noalloc_matches_the_allocating_call_twice_in_a_row(ctx):
    big = inputs.rmat(21, 8 << 21, 0.57, 0.19, 0.19, seed=21)      # 2^21 vertices: ~43 MiB of workspace
    small = inputs.disjoint_union([inputs.er(30_000, 90_000, seed=22), inputs.chain(777, seed=23),
                                   inputs.empty(5)])
    graphs = []
    for g in (big, small):
        d = b.build_csr(ctx, g.n, g.u, g.v)
        want, wc = oracle.uf_cc(g.n, g.u, g.v)
        graphs.append((g, d, want, wc))
    assert b.workspace_bytes(big.n, graphs[0][1].m, b.default_variant()) <= b.noalloc_scratch_bytes()
    dev = ctx.torch_device
    for v in _variants():
        for g, d, want, wc in graphs:                                   # large first, then smaller
            print(f"[noalloc] {g} {v.name()}", file=sys.stderr, flush=True)
            lab_a, nc_a = b.connectivity_csr(ctx, d, v)
            lab_n = torch.full((g.n,), -7, dtype=torch.int32, device=dev)
            nc_n = torch.full((1,), -7, dtype=torch.int64, device=dev)
            b.connectivity_csr_noalloc(ctx, d, v, labels=lab_n, ncomp=nc_n)
            torch.cuda.synchronize()
            ctx.sync_status()
            got = lab_n.cpu().numpy()
            assert np.array_equal(got, lab_a.cpu().numpy()), v.name()
            assert int(nc_n.item()) == int(nc_a.item()) == wc, v.name()
            assert np.array_equal(got, want), v.name()


def test_noalloc_with_timing_on_records_nothing(ctx):
    g = inputs.er(20_000, 60_000, seed=24)
    d = b.build_csr(ctx, g.n, g.u, g.v)
    want, wc = oracle.uf_cc(g.n, g.u, g.v)
    ctx.set_timing(True)
    ctx.phase_times_reset()
    lab, nc = b.connectivity_csr_noalloc(ctx, d)
    torch.cuda.synchronize()
    assert ctx.phase_times() == {}
    ctx.set_timing(False)
    assert np.array_equal(lab.cpu().numpy(), want) and int(nc.item()) == wc


def test_noalloc_refuses_graphs_beyond_the_array(ctx):
    n = 1 << 22                                                       # all isolated: a valid CSR
    dev = ctx.torch_device
    d = b.CSR(n, torch.zeros(n + 1, dtype=torch.int32, device=dev), torch.zeros(1, dtype=torch.int32, device=dev)[:0])
    assert b.workspace_bytes(n, 0, b.default_variant()) > b.noalloc_scratch_bytes()
    with pytest.raises(b.CCError) as ei:
        b.connectivity_csr_noalloc(ctx, d)
    assert ei.value.status == b.CC_ENOMEM and "no-allocation" in str(ei.value)
    ctx.sync_status()
