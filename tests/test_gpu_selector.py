"""Selector kernels against the CPU oracle: BF16 MLP forward / backward /
Adam, graph features, and the automatic entry point (which must return the
oracle's labels whatever arm it picks)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp
from paper_2008_03909_amd import binding as b
from paper_2008_03909_amd import inputs, selector

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = b.Context(0)
    yield c
    c.close()


def _bf16_bits(x):
    """BF16 bit patterns (int16) of float values, and the rounded values."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    return u.view(np.int16), omlp.bf16_round(f)


@pytest.mark.parametrize("K,B", [(16, 1), (16, 37), (3, 64), (100, 5)])
def test_mlp_forward_and_backward_match_oracle(ctx, K, B):
    rng = np.random.default_rng(K * 100 + B)
    dev = ctx.torch_device
    bits, pv = _bf16_bits(rng.normal(0, 0.25, omlp.param_count(K)))
    X = rng.normal(0, 1, (B, 16)).astype(np.float32)
    T = rng.normal(0, 1, (B, K)).astype(np.float32)
    P = torch.from_numpy(bits).to(dev)
    Xd = torch.from_numpy(X).to(dev)
    cache = torch.empty(B * 256, dtype=torch.float32, device=dev)
    Y = b.mlp_forward(P, K, Xd, cache).cpu().numpy()
    want, _ = omlp.forward(pv, X.astype(np.float64), K)
    assert np.max(np.abs(Y - want)) <= 1e-2 * max(1.0, np.max(np.abs(want)))
    g, loss = b.mlp_backward(P, K, Xd, cache, torch.from_numpy(Y).to(dev), torch.from_numpy(T).to(dev))
    wl, wg = omlp.loss_and_grads(pv, X.astype(np.float64), T.astype(np.float64), K)
    g = g.cpu().numpy()
    # per parameter block: relative Frobenius error
    sizes = [16 * 64, 64, 64 * 64, 64, 64 * K, K]
    o = 0
    for s in sizes:
        num = np.linalg.norm(g[o:o + s] - wg[o:o + s])
        den = max(np.linalg.norm(wg[o:o + s]), 1e-12)
        assert num <= 2e-2 * den or np.linalg.norm(wg[o:o + s]) < 1e-9
        o += s
    assert abs(float(loss.item()) - wl) <= 1e-2 * max(wl, 1e-6)


def test_mlp_adam_matches_oracle(ctx):
    rng = np.random.default_rng(4)
    dev = ctx.torch_device
    n = 1000
    w = rng.normal(0, 1, n).astype(np.float32)
    m1 = np.zeros(n)
    m2 = np.zeros(n)
    master = torch.from_numpy(w.copy()).to(dev)
    params = torch.empty(n, dtype=torch.int16, device=dev)
    dm1 = torch.zeros(n, dtype=torch.float32, device=dev)
    dm2 = torch.zeros(n, dtype=torch.float32, device=dev)
    ww = w.astype(np.float64)
    for step in range(1, 6):
        g = rng.normal(0, 1, n).astype(np.float32)
        b.mlp_adam(master, params, torch.from_numpy(g).to(dev), dm1, dm2, 1e-2, 0.9, 0.999, 1e-8, step)
        ww, m1, m2 = omlp.adam_step(ww, g.astype(np.float64), m1, m2, 1e-2, 0.9, 0.999, 1e-8, step)
    assert np.allclose(master.cpu().numpy(), ww, rtol=1e-4, atol=1e-5)
    bits, _ = _bf16_bits(master.cpu().numpy())
    assert np.array_equal(params.cpu().numpy(), bits)


def test_graph_features_match_oracle(ctx):
    gs = [inputs.er(5000, 30000, seed=1), inputs.grid(2, 60, 0.7, seed=2),
          inputs.disjoint_union([inputs.star(300), inputs.chain(400, seed=3), inputs.empty(50)]),
          inputs.rmat(13, 8 << 13, 0.57, 0.19, 0.19, seed=4), inputs.path(3000), inputs.clique(40),
          inputs.star(9000, 5), inputs.empty(64), inputs.grid(3, 18, 0.5, seed=5)]
    seed = b.default_variant().seed
    for g in gs:
        d = b.build_csr(ctx, g.n, g.u, g.v)
        feats = b.graph_features(ctx, d)
        off, adj = oracle.csr_build(g.n, g.u, g.v, True)
        want = oracle.degree_features(off)
        want.update(oracle.sampled_features(g.n, off, adj, seed))
        assert sorted(want) == list(range(16))
        for i, w in want.items():
            assert abs(feats[i] - w) <= 1e-4 * max(1.0, abs(w)), (g, i, feats[i], w)
        # the probes' level and reached totals are integers: exact
        assert round(feats[12] * 16) == round(want[12] * 16), g
        assert round(feats[13] * g.n * 16) == round(want[13] * g.n * 16), g


def test_auto_returns_oracle_labels_for_every_arm(ctx):
    arms = selector.arms()
    K = len(arms)
    g = inputs.disjoint_union([inputs.er(3000, 9000, seed=5), inputs.grid(2, 30, 0.6, seed=6)])
    want, wc = oracle.labels(g)
    d = b.build_csr(ctx, g.n, g.u, g.v)
    norm = np.concatenate([np.zeros(16), np.ones(16)]).astype(np.float32)
    dev = ctx.torch_device
    seen = set()
    for j in range(K):
        # a model whose output bias makes arm j the unique argmin
        master = np.zeros(b.mlp_param_count(K), np.float32)
        master[-K:] = 1.0
        master[-K + j] = -1.0
        params = b.mlp_pack_bf16(torch.from_numpy(master).to(dev))
        lab, nc, chosen, feats = b.connectivity_auto(ctx, d, params, arms, norm)
        assert chosen == j
        seen.add(chosen)
        assert int(nc.item()) == wc and np.array_equal(lab.cpu().numpy(), want), arms[j]
    lab, nc, chosen, _ = b.connectivity_auto(ctx, d, None, None, None)
    assert chosen == -1 and np.array_equal(lab.cpu().numpy(), want)
    assert seen == set(range(K))


def test_select_variant_agrees_with_auto(ctx):
    arms = selector.arms()
    K = len(arms)
    g = inputs.rmat(12, 8 << 12, 0.6, 0.175, 0.175, seed=11)
    d = b.build_csr(ctx, g.n, g.u, g.v)
    norm = np.concatenate([np.zeros(16), np.ones(16)]).astype(np.float32)
    dev = ctx.torch_device
    for j in (0, 7, K - 1):
        master = np.zeros(b.mlp_param_count(K), np.float32)
        master[-K:] = 1.0
        master[-K + j] = -1.0
        params = b.mlp_pack_bf16(torch.from_numpy(master).to(dev))
        var, chosen, feats = b.select_variant(ctx, d, params, arms, norm)
        assert chosen == j and var.name() == arms[j].name()
        _, _, chosen2, feats2 = b.connectivity_auto(ctx, d, params, arms, norm)
        assert chosen2 == j and feats == feats2
    var, chosen, _ = b.select_variant(ctx, d, None, None, None)
    assert chosen == -1 and var.name() == b.default_variant().name()


def test_training_lowers_the_loss(ctx):
    rng = np.random.default_rng(0)
    N, K = 256, 16
    X = rng.normal(0, 1, (N, 16)).astype(np.float32)
    W = rng.normal(0, 1, (16, K))
    Y = np.maximum(X @ W, 0).astype(np.float32) * 0.3
    _, _, hist = selector.train(ctx, X, Y, epochs=60, batch=32, lr=3e-3)
    assert hist[-1] < 0.5 * hist[0]


def test_decision_matches_oracle_forward_with_the_trained_model(ctx):
    """The device decision (forward pass and argmin on the returned features)
    equals the oracle's forward pass on the same features, unless the two
    best outputs are within rounding of each other."""
    import os
    z = np.load(os.path.join(os.path.dirname(selector.__file__), "selector_data", "model.npz"), allow_pickle=False)
    K, norm = int(z["K"]), z["norm"].astype(np.float32)
    params = b.mlp_pack_bf16(torch.from_numpy(z["master"].astype(np.float32)).to(ctx.torch_device))
    arms = selector.arms()
    sd = np.where(norm[16:] > 0, norm[16:], 1.0).astype(np.float32)
    checked = 0
    for s in (1000, 1010, 1020, 1030, 1040, 1050, 1060, 1070):
        fam, g = selector.corpus_graph(s, 12, 16)
        d = b.build_csr(ctx, g.n, g.u, g.v)
        _, chosen, feats = b.select_variant(ctx, d, params, arms, norm)
        x = (np.array(feats, np.float32) - norm[:16]) / sd
        y, _ = omlp.forward(omlp.bf16_round(z["master"]), x[None, :].astype(np.float64), K)
        y = y[0]
        order = np.argsort(y, kind="stable")
        if y[order[1]] - y[order[0]] > 1e-3 * max(1.0, abs(y[order[0]])):
            assert chosen == int(order[0]), (fam, s, chosen, order[:2])
            checked += 1
        else:
            assert chosen in (int(order[0]), int(order[1])), (fam, s)
    assert checked >= 4
