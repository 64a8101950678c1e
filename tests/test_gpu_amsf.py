"""Approximate minimum spanning forest (Section 5.1) against the oracle.

A (1 + eps) forest is not unique, so the edges are checked rather than
compared: every returned pair is an adjacency entry, none closes a cycle,
the forest connects what the graph connects (labels equal the oracle's) and
has n - c edges, each returned weight is the weight of its edge, and the
number of forest edges in each weight bucket equals the oracle's bucketed
Kruskal count (the same for every forest the method can return; the
buckets are decided in float on both sides).  The total weight is at most
(1 + eps) times the exact minimum (the oracle's Kruskal)."""
import sys

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


def _note(msg):
    print(f"[amsf] {msg}", file=sys.stderr, flush=True)


def _host_csr(d):
    off = d.offsets.cpu().numpy().astype(np.int64)
    adj = d.adj.cpu().numpy()
    rows = np.repeat(np.arange(d.n, dtype=np.int32), np.diff(off))
    return off, adj, rows


def _check(ctx, d, w, opt, name, want=None, rows_adj=None):
    """Runs cc_amsf_csr on device CSR d with per-entry weights w (host
    float32) and checks it against the oracle."""
    off, adj, rows = rows_adj if rows_adj is not None else _host_csr(d)
    dev = ctx.torch_device
    wt = torch.from_numpy(w).to(dev)
    out = b.amsf_csr(ctx, d, wt, opt)
    torch.cuda.synchronize()
    ctx.sync_status()
    _verify(d.n, d.m, off, adj, rows, w, opt, name, out, want)


def _verify(n, m, off, adj, rows, w, opt, name, out, want=None):
    """The oracle's checks of one result on the host CSR (off, adj, rows)
    with entry weights w."""
    lab, eu, ev, ew, ne, tw = out
    k = int(ne.item())
    fu, fv, fw = eu[:k].cpu().numpy(), ev[:k].cpu().numpy(), ew[:k].cpu().numpy()
    if want is None:
        want = oracle.uf_cc(n, rows, adj)
    wl, wc = want
    assert np.array_equal(lab.cpu().numpy(), wl), name
    assert k == n - wc, (name, k, n - wc)
    assert oracle.forest_check_csr(n, off, adj, wl, fu, fv) == oracle.FOREST_OK, name
    # each returned weight is its edge's weight (entry weights are a function of the pair)
    key = rows.astype(np.int64) * n + adj
    order = np.argsort(key, kind="stable")
    pos = np.searchsorted(key[order], fu.astype(np.int64) * n + fv)
    assert np.array_equal(fw, w[order][pos]), name
    if m == 0:
        assert k == 0 and float(tw.item()) == 0.0
        return
    t, cnt = oracle.amsf_buckets(n, rows, adj, w, opt.epsilon)
    fb = np.searchsorted(t, fw, side="right") - 1
    assert np.array_equal(np.bincount(fb, minlength=len(cnt)), cnt), name
    exact, ek = oracle.msf_weight(n, rows, adj, w.astype(np.float64))
    assert ek == k
    total = float(tw.item())
    assert abs(total - float(np.sum(fw, dtype=np.float64))) <= 1e-9 * max(total, 1.0), name
    assert total <= (1.0 + opt.epsilon) * exact * (1 + 1e-9), (name, total, exact)
    assert total >= exact * (1 - 1e-9), (name, total, exact)


def _weights_for(d, seed, mean=1.0):
    off, adj, rows = _host_csr(d)
    return inputs.pair_weights(d.n, rows, adj, seed, mean), (off, adj, rows)


@pytest.mark.parametrize("lf", [0.0, 0.125, 0.5, 1.0])
def test_amsf_suite(ctx, lf):
    opt = b.amsf_options(light_fraction=lf)
    for i, g in enumerate(SUITE):
        d = b.build_csr(ctx, g.n, g.u, g.v)
        w, ra = _weights_for(d, seed=100 + i)
        _note(f"{g} lf={lf}")
        _check(ctx, d, w, opt, f"{g} lf={lf}", rows_adj=ra)


@pytest.mark.parametrize("eps", [0.01, 0.1, 1.0, 8.0])
def test_amsf_epsilons(ctx, eps):
    g = inputs.rmat(14, 8 << 14, 0.57, 0.19, 0.19, seed=21)
    d = b.build_csr(ctx, g.n, g.u, g.v)
    w, ra = _weights_for(d, seed=22)
    for lf in (0.0, 0.125):
        _check(ctx, d, w, b.amsf_options(epsilon=eps, light_fraction=lf), f"eps={eps} lf={lf}", rows_adj=ra)


def test_amsf_int64_offsets_and_seeds(ctx):
    g = inputs.er(20000, 120000, seed=31)
    d = b.build_csr(ctx, g.n, g.u, g.v, offsets_64bit=True)
    assert d.o64
    w, ra = _weights_for(d, seed=32)
    for seed in (1, 2, 3):
        _check(ctx, d, w, b.amsf_options(seed=seed, light_fraction=0.25), f"o64 seed={seed}", rows_adj=ra)


def test_amsf_equal_and_tied_weights(ctx):
    # every weight equal: one bucket; weights on bucket boundaries
    g = inputs.grid(2, 50, 0.7, seed=41)
    d = b.build_csr(ctx, g.n, g.u, g.v)
    off, adj, rows = _host_csr(d)
    _check(ctx, d, np.full(d.m, 2.5, np.float32), b.amsf_options(), "equal", rows_adj=(off, adj, rows))
    lo = np.minimum(rows, adj).astype(np.int64)
    hi = np.maximum(rows, adj).astype(np.int64)
    w = (1.25 ** ((lo * 7 + hi * 3) % 9)).astype(np.float32)  # exact bucket boundaries at eps = 0.25
    for lf in (0.0, 0.3):
        _check(ctx, d, w, b.amsf_options(light_fraction=lf), f"boundaries lf={lf}", rows_adj=(off, adj, rows))


def test_amsf_self_loops_and_wide_range(ctx):
    # a hand-made CSR with self-loop entries (one holding the minimum weight)
    # and weights over 30 orders of magnitude
    n = 6
    rows_l = [[0, 0, 1], [0, 2], [1, 2, 2], [4], [3], [5]]  # rows sorted; self-loops on 0, 2 and 5
    off = np.zeros(n + 1, np.int32)
    off[1:] = np.cumsum([len(r) for r in rows_l])
    adj = np.array([x for r in rows_l for x in r], np.int32)
    rows = np.repeat(np.arange(n, dtype=np.int32), np.diff(off))
    pw = {(0, 0): 1e-20, (0, 1): 3e-5, (1, 2): 2e10, (2, 2): 1.0, (3, 4): 0.5, (5, 5): 4.0}
    w = np.array([pw[(min(a, c), max(a, c))] for a, c in zip(rows, adj)], np.float32)
    dev = ctx.torch_device
    d = b.CSR(n, torch.from_numpy(off).to(dev), torch.from_numpy(adj).to(dev))
    for lf in (0.0, 0.5, 1.0):
        _check(ctx, d, w, b.amsf_options(light_fraction=lf), f"loops lf={lf}",
               rows_adj=(off.astype(np.int64), adj, rows))


def test_amsf_empty_graph(ctx):
    dev = ctx.torch_device
    d = b.CSR(9, torch.zeros(10, dtype=torch.int32, device=dev), torch.zeros(0, dtype=torch.int32, device=dev))
    lab, eu, ev, ew, ne, tw = b.amsf_csr(ctx, d, torch.zeros(0, dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    assert int(ne.item()) == 0 and float(tw.item()) == 0.0
    assert np.array_equal(lab.cpu().numpy(), np.arange(9))


def test_amsf_rejects_bad_input(ctx):
    g = inputs.er(500, 2000, seed=51)
    d = b.build_csr(ctx, g.n, g.u, g.v)
    dev = ctx.torch_device
    w, _ = _weights_for(d, seed=52)
    for bad in (0.0, -1.0, np.nan, np.inf):
        x = w.copy()
        x[d.m // 2] = bad
        with pytest.raises(b.CCError):
            b.amsf_csr(ctx, d, torch.from_numpy(x).to(dev))
    for opt in (b.amsf_options(epsilon=0.0), b.amsf_options(epsilon=1e-9), b.amsf_options(light_fraction=1.5)):
        with pytest.raises(b.CCError):
            b.amsf_csr(ctx, d, torch.from_numpy(w).to(dev), opt)
    # a weight range that needs more than 4096 buckets at this epsilon
    x = w.copy()
    x[0] = 1e-30
    x[1] = 1e30
    with pytest.raises(b.CCError):
        b.amsf_csr(ctx, d, torch.from_numpy(x).to(dev), b.amsf_options(epsilon=0.01))
    # the context still works afterwards
    _check(ctx, d, w, b.amsf_options(), "after errors")


@pytest.mark.parametrize("lf", [0.0, 0.5])
def test_amsf_mapped_suite(ctx, lf):
    """On the degree-ordered CSR, with each entry weighted as the same pair of
    original vertices: edges, weights and labels come back in the original
    numbering and pass the checks on the original CSR."""
    opt = b.amsf_options(light_fraction=lf)
    for i, g in enumerate(SUITE):
        d0 = b.build_csr(ctx, g.n, g.u, g.v)
        w0, ra = _weights_for(d0, seed=100 + i)
        r = b.build_csr_degree_order(ctx, g.n, g.u, g.v)
        off_r, adj_r, rows_r = _host_csr(r)
        orig = r.orig_of.cpu().numpy()
        wr = inputs.pair_weights(g.n, orig[rows_r], orig[adj_r], 100 + i, 1.0)
        _note(f"{g} mapped lf={lf}")
        out = b.amsf_csr_mapped(ctx, r, torch.from_numpy(wr).to(ctx.torch_device), opt)
        torch.cuda.synchronize()
        ctx.sync_status()
        _verify(g.n, d0.m, ra[0], ra[1], ra[2], w0, opt, f"{g} mapped lf={lf}", out)

