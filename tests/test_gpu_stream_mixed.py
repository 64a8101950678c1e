"""Mixed batches (the streaming appendix's ProcessBatch; Section 3.4's
three types of streaming algorithms) against the oracle.

Within a batch, a query may be linearized before or after each concurrent
insert, so its answer is checked against the two bounds the oracle fixes:
1 if its endpoints were connected before the batch, 0 if they are not
connected after it.  Type-2 and type-3 streams run the batch's inserts
before its queries, so their answers must equal the after-batch state.
After every batch the stream's labels equal the oracle's."""
import numpy as np
import pytest
import torch

import oracle
from paper_2008_03909_amd import binding as b

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = b.Context(0)
    yield c
    c.close()


def _variants():
    vs = [b.default_variant(finish=fin, find=f) for fin in (b.FIN_UF_ASYNC, b.FIN_UF_EARLY, b.FIN_UF_HOOKS)
          for f in range(4)]
    vs += [b.default_variant(finish=b.FIN_UF_REM_CAS, splice=s, find=f) for s in range(3) for f in range(3)]
    vs += [b.default_variant(finish=b.FIN_SV)]
    vs += [b.default_variant(finish=b.FIN_LT, lt_rules=r) for r in (b.LT_CRSA, b.LT_PRSA, b.LT_PRS, b.LT_CRFA, b.LT_PRFA, b.LT_PRF)]
    return vs


def _expected_type(v):
    if v.finish in (b.FIN_SV, b.FIN_LT):
        return 2
    if v.finish == b.FIN_UF_REM_CAS and v.splice == b.SPLICE_ATOMIC:
        return 3
    return 1


def _batch(rng, n, k, pending):
    """k operations, about half inserts; many queries ask about the
    endpoints of this batch's own inserts (answers that depend on the
    linearization), the rest are uniform."""
    kind = (rng.random(k) < 0.5).astype(np.uint8)
    u = rng.integers(0, n, k).astype(np.int32)
    v = rng.integers(0, n, k).astype(np.int32)
    ins = np.flatnonzero(kind == 0)
    qs = np.flatnonzero(kind == 1)
    if ins.size and qs.size:
        pick = rng.integers(0, ins.size, qs.size)
        near = rng.random(qs.size) < 0.5
        # query the inserted edge's endpoints, or one endpoint and a vertex a
        # prior batch touched
        u[qs[near]] = u[ins[pick[near]]]
        v[qs[near]] = v[ins[pick[near]]]
        if pending.size:
            v[qs[~near]] = pending[rng.integers(0, pending.size, int((~near).sum()))]
    return kind, u, v


@pytest.mark.parametrize("vi", range(len(_variants())))
def test_mixed_batches_are_linearizable(ctx, vi):
    v = _variants()[vi]
    n = 4000
    st = b.Stream(ctx, n, v)
    assert st.type == _expected_type(v)
    inc = oracle.Incremental(n)
    rng = np.random.default_rng(100 + vi)
    dev = ctx.torch_device
    touched = np.zeros(0, np.int32)
    undecided = 0
    for batch in range(10):
        k = int(rng.integers(1, 6000))
        kind, u, w = _batch(rng, n, k, touched)
        qs = kind != 0
        before = inc.query(u[qs], w[qs])
        got = st.process(torch.from_numpy(kind).to(dev), torch.from_numpy(u).to(dev),
                         torch.from_numpy(w).to(dev)).cpu().numpy()
        inc.insert(u[~qs], w[~qs])
        after = inc.query(u[qs], w[qs])
        ans = got[qs]
        assert np.all(got[~qs] == 0), (v, batch)
        assert np.all(ans[before == 1] == 1), (v, batch)
        assert np.all(ans[after == 0] == 0), (v, batch)
        if st.type != 1:
            assert np.array_equal(ans, after), (v, batch)
        undecided += int(((before == 0) & (after == 1)).sum())
        lab, nc = st.labels()
        want, wc = inc.labels()
        assert np.array_equal(lab.cpu().numpy(), want) and int(nc.item()) == wc, (v, batch)
        touched = np.unique(np.concatenate([touched, u[~qs], w[~qs]])).astype(np.int32)
    assert undecided > 0  # the batches did exercise queries whose answer depends on the order
    st.sync_status()
    st.close()


def test_mixed_batch_edge_cases(ctx):
    dev = ctx.torch_device
    for v in (b.default_variant(finish=b.FIN_UF_ASYNC), b.default_variant(finish=b.FIN_SV),
              b.default_variant(splice=b.SPLICE_ATOMIC), b.default_variant(finish=b.FIN_UF_HOOKS)):
        st = b.Stream(ctx, 10, v)
        # empty batch, self-loops, a query on one vertex, repeated pairs
        st.process(torch.zeros(0, dtype=torch.uint8, device=dev), torch.zeros(0, dtype=torch.int32, device=dev),
                   torch.zeros(0, dtype=torch.int32, device=dev))
        kind = np.array([0, 0, 1, 1, 0, 1], np.uint8)
        u = np.array([3, 3, 3, 4, 1, 2], np.int32)
        w = np.array([3, 4, 3, 3, 2, 1], np.int32)
        got = st.process(kind, u, w).cpu().numpy()
        assert got[2] == 1 and got[0] == 0 and got[1] == 0 and got[4] == 0
        assert got[3] in (0, 1) and got[5] in (0, 1)
        lab, _ = st.labels()
        assert lab.cpu().numpy().tolist() == [0, 1, 1, 3, 3, 5, 6, 7, 8, 9]
        # out-of-range ids: skipped, reported through the error word
        st.process(np.array([0, 1], np.uint8), np.array([0, 11], np.int32), np.array([12, 0], np.int32))
        with pytest.raises(b.CCError):
            st.sync_status()
        lab, _ = st.labels()
        assert lab.cpu().numpy().tolist() == [0, 1, 1, 3, 3, 5, 6, 7, 8, 9]
        st.close()


def test_type2_stream_initialize_then_batches(ctx):
    # Initialize(G) with the static SV / LT run, then mixed batches in rounds
    from paper_2008_03909_amd import inputs
    g = inputs.er(3000, 2000, seed=9)
    dev = ctx.torch_device
    d = b.build_csr(ctx, g.n, g.u, g.v)
    for v in (b.default_variant(finish=b.FIN_SV, sample=b.SAMPLE_NONE),
              b.default_variant(finish=b.FIN_LT, lt_rules=b.LT_PRFA)):
        st = b.Stream(ctx, g.n, v)
        st.init_csr(d, v)
        inc = oracle.Incremental(g.n)
        inc.insert(g.u, g.v)
        rng = np.random.default_rng(5)
        for _ in range(4):
            kind, u, w = _batch(rng, g.n, 3000, np.zeros(0, np.int32))
            qs = kind != 0
            got = st.process(kind, u, w).cpu().numpy()
            inc.insert(u[~qs], w[~qs])
            assert np.array_equal(got[qs], inc.query(u[qs], w[qs]))
        lab, _ = st.labels()
        assert np.array_equal(lab.cpu().numpy(), inc.labels()[0])
        st.close()


def test_non_streaming_finishes_are_refused(ctx):
    for v in (b.default_variant(finish=b.FIN_LP), b.default_variant(finish=b.FIN_LT, lt_rules=b.LT_NONROOT["PUS"])):
        with pytest.raises(b.CCError):
            b.Stream(ctx, 10, v)


@pytest.mark.parametrize("fin,rules", [(b.FIN_SV, 0), (b.FIN_LT, b.LT_CRSA), (b.FIN_LT, b.LT_PRF)])
def test_type2_batch_larger_than_the_edge_list(ctx, fin, rules):
    """A type-2 stream keeps a fixed edge list of 2^22 pairs and inserts a
    larger batch as consecutive parts: one insert batch of 5,000,000 pairs
    (plus a mixed batch of 4,500,000 operations) gives the oracle's labels,
    and the mixed batch's queries see all of its inserts."""
    n = 1 << 20
    rng = np.random.default_rng(31)
    u = rng.integers(0, n, 5_000_000).astype(np.int32)
    v = rng.integers(0, n, 5_000_000).astype(np.int32)
    u[:1000] = v[:1000]                       # self-loops are no-ops
    st = b.Stream(ctx, n, b.default_variant(finish=fin, lt_rules=rules or b.LT_PRF))
    assert st.type == 2
    dev = ctx.torch_device
    st.insert(torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev))
    lab, nc = st.labels()
    torch.cuda.synchronize()
    want, wc = oracle.uf_cc(n, u, v)
    assert np.array_equal(lab.cpu().numpy(), want) and int(nc.item()) == wc
    k = 4_500_000
    kind = (rng.random(k) < 0.5).astype(np.uint8)
    a = rng.integers(0, n, k).astype(np.int32)
    c = rng.integers(0, n, k).astype(np.int32)
    out = st.process(kind, a, c).cpu().numpy()
    st.sync_status()
    ins = kind == 0
    want2, _ = oracle.uf_cc(n, np.concatenate([u, a[ins]]), np.concatenate([v, c[ins]]))
    q = ~ins
    assert np.array_equal(out[q], (want2[a[q]] == want2[c[q]]).astype(np.uint8))
    assert not out[ins].any()
    lab2, _ = st.labels()
    assert np.array_equal(lab2.cpu().numpy(), want2)
    st.close()
