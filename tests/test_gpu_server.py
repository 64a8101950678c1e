"""Serving loop: continuous batching gives every request the answer it gets
alone -- the oracle's answer against exactly the inserts that arrived before
it -- whatever the mix, the number of streams and the memory budget."""
import numpy as np
import pytest

import oracle
from paper_2008_03909_amd import binding as b
from paper_2008_03909_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = b.Context(0)
    yield c
    c.close()


def _trace(n, count, seed, max_insert=20000, max_query=5000):
    """Alternating-ish random request mix over an R-MAT-like edge stream."""
    rng = np.random.default_rng(seed)
    g = inputs.rmat(int(np.log2(n)), 4 * n, 0.57, 0.19, 0.19, seed=seed)
    eu, ev = inputs.shuffle_pairs(g.u, g.v, seed)
    types, starts, lens, A, B = [], [], [], [], []
    pos_e, pos = 0, 0
    for i in range(count):
        t = int(rng.random() < 0.5)
        if t == 0:
            k = int(min(inputs.log_uniform_int(10, max_insert, rng.random()), eu.size - pos_e))
            if k <= 0:
                t = 1
            else:
                A.append(eu[pos_e:pos_e + k])
                B.append(ev[pos_e:pos_e + k])
                pos_e += k
        if t == 1:
            k = inputs.log_uniform_int(10, max_query, rng.random())
            qa, qb = inputs.query_pairs(n, k, seed=seed * 1000 + i)
            A.append(qa)
            B.append(qb)
        types.append(t)
        starts.append(pos)
        lens.append(k)
        pos += k
    return (np.array(types, np.int32), np.array(starts, np.int64), np.array(lens, np.int64),
            np.concatenate(A).astype(np.int32), np.concatenate(B).astype(np.int32))


def _alone(n, types, starts, lens, A, B):
    """Each query answered alone: the oracle after exactly the earlier inserts."""
    inc = oracle.Incremental(n)
    out = np.zeros(A.size, np.uint8)
    for t, s, k in zip(types, starts, lens):
        sl = slice(s, s + k)
        if t == 0:
            inc.insert(A[sl], B[sl])
        else:
            out[sl] = inc.query(A[sl], B[sl])
    return out


BARRIER_VARIANT = b.default_variant(finish=b.FIN_UF_REM_CAS, splice=b.SPLICE_SPLIT_ONE, find=b.FIND_NAIVE)


@pytest.mark.parametrize("streams,budget,variant", [(1, 1 << 24, None), (4, 1 << 24, None), (8, 1 << 20, None),
                                                    (4, 1 << 24, BARRIER_VARIANT)])
def test_server_submit_matches_alone(ctx, streams, budget, variant):
    n = 1 << 15
    types, starts, lens, A, B = _trace(n, 120, seed=streams)
    srv = b.Server(ctx, n, variant=variant, budget_bytes=budget, num_streams=streams, max_inflight=32)
    assert srv.stamped == (variant is None)
    outs = []
    for t, s, k in zip(types, starts, lens):
        sl = slice(s, s + k)
        if t == 0:
            srv.insert(A[sl], B[sl])
        else:
            outs.append((sl, srv.query(A[sl], B[sl])[1]))
        srv.poll()
    srv.poll(wait_all=True)
    want = _alone(n, types, starts, lens, A, B)
    for sl, o in outs:
        assert np.array_equal(o, want[sl])
    assert srv.pool_used() == 0
    lab, _ = srv.labels()
    inc = oracle.Incremental(n)
    for t, s, k in zip(types, starts, lens):
        if t == 0:
            inc.insert(A[s:s + k], B[s:s + k])
    assert np.array_equal(lab.cpu().numpy(), inc.labels()[0])
    srv.close()


def _pinned(x):
    """A numpy view of a pinned (device-mapped) host copy of x."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).pin_memory()
    return t.numpy(), t


@pytest.mark.parametrize("variant,pinned", [(None, False), (BARRIER_VARIANT, False), (None, True),
                                            (BARRIER_VARIANT, True)])
def test_server_trace_in_the_mix_equals_alone(ctx, variant, pinned):
    """Poisson arrivals fast enough that requests overlap on the device (in
    stamped mode queries also overlap the inserts that arrive after them).
    Pageable payloads are copied through the pool; pinned ones are read and
    answered in place by the kernels."""
    n = 1 << 16
    types, starts, lens, A, B = _trace(n, 300, seed=7, max_insert=200000, max_query=50000)
    rng = np.random.default_rng(3)
    arrivals = np.cumsum(rng.exponential(20e-6, types.size))
    # in place, requests need no pool: a 64 KiB budget would refuse most of
    # them as copies (up to 200,000 pairs, 1.6 MB)
    srv = b.Server(ctx, n, variant=variant, budget_bytes=(1 << 16) if pinned else (1 << 26), num_streams=2,
                   max_inflight=16)
    if pinned:
        (pa, ta), (pb, tb), (po, to) = _pinned(A), _pinned(B), _pinned(np.zeros(A.size, np.uint8))
        got, lat = srv.run_trace(types, arrivals, starts, lens, pa, pb, po)
    else:
        got, lat = srv.run_trace(types, arrivals, starts, lens, A, B)
    want = _alone(n, types, starts, lens, A, B)
    q = np.zeros(A.size, bool)
    for t, s, k in zip(types, starts, lens):
        if t == 1:
            q[s:s + k] = True
    assert np.array_equal(got[q], want[q])
    assert np.all(lat > 0)
    srv.close()


def test_server_rejects_requests_over_budget(ctx):
    srv = b.Server(ctx, 1000, budget_bytes=4096, num_streams=2, max_inflight=4)
    big = np.zeros(1000, np.int32)
    with pytest.raises(b.CCError) as ei:
        srv.insert(big, big)
    assert ei.value.status == b.CC_EBUSY
    # requests that fit are admitted one at a time and still answer correctly
    u = np.arange(0, 400, dtype=np.int32)
    v = np.arange(1, 401, dtype=np.int32)
    srv.insert(u, v)
    rid, out = srv.query(np.array([0, 0, 500], np.int32), np.array([400, 401, 0], np.int32))
    srv.poll(wait_all=True)
    assert out.tolist() == [1, 0, 0]
    assert srv.info(rid)[0]
    srv.close()


def test_server_state_stays_bounded_and_answers_stay_exact(ctx):
    """3,000 small requests that alternate between inserts and queries (a
    phase change at almost every request): every answer equals the alone
    answer, the HIP events the server holds stay bounded by the requests in
    flight, and the outcome of recent requests is still reported."""
    n = 1 << 14
    types, starts, lens, A, B = _trace(n, 3000, seed=11, max_insert=300, max_query=300)
    srv = b.Server(ctx, n, budget_bytes=1 << 22, num_streams=4, max_inflight=8)
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(2e-6, types.size))
    got, lat = srv.run_trace(types, arrivals, starts, lens, A, B)
    want = _alone(n, types, starts, lens, A, B)
    q = np.zeros(A.size, bool)
    for t, s0, k in zip(types, starts, lens):
        if t == 1:
            q[s0:s0 + k] = True
    assert np.array_equal(got[q], want[q])
    assert np.all(lat > 0)
    # two per request in flight (completion, payload copy) and the barriers
    # of the phases those requests belong to
    assert srv.event_count() <= 3 * 8 + 1, srv.event_count()
    rid = srv.insert(np.array([1], np.int32), np.array([2], np.int32))
    srv.poll(wait_all=True)
    done, l1 = srv.info(rid)
    assert done and l1 > 0
    assert srv.pool_used() == 0
    srv.close()


def test_server_labels_after_stamped_inserts(ctx):
    """The stamped state's labels (every link, whatever its phase) equal the
    oracle's labels of all inserts, and bad ids are reported."""
    n = 5000
    g = inputs.er(n, 4000, seed=12)
    srv = b.Server(ctx, n, budget_bytes=1 << 20, num_streams=2, max_inflight=4)
    for i in range(0, g.u.size, 700):
        srv.insert(g.u[i:i + 700], g.v[i:i + 700])
        srv.query(g.u[:50], g.v[::-1][:50])
    lab, nc = srv.labels()
    want, wc = oracle.uf_cc(n, g.u, g.v)
    assert np.array_equal(lab.cpu().numpy(), want) and int(nc.item()) == wc
    srv.insert(np.array([3, n + 5], np.int32), np.array([4, 1], np.int32))
    with pytest.raises(b.CCError):
        srv.poll(wait_all=True)
    srv.close()
