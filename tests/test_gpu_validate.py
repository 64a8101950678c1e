"""The CSR validator (cc_validate_csr) against the oracle's checker on
planted defects, with 32- and 64-bit offsets, and on the full-size R-MAT
2^24 CSR.  Only the validator ever sees a malformed CSR: no connectivity
kernel runs on one."""
import sys

import numpy as np
import pytest
import torch

import csr_cases
import oracle
from paper_2008_03909_amd import binding as b
from paper_2008_03909_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = b.Context(0)
    yield c
    c.close()


def _dev_csr(ctx, c, o64):
    dev = ctx.torch_device
    off = torch.from_numpy(c.off.astype(np.int64 if o64 else np.int32)).to(dev)
    adj = torch.from_numpy(c.adj if len(c.adj) else np.zeros(1, np.int32)).to(dev)
    g = b.CSR(c.n, off, adj[:len(c.adj)] if len(c.adj) else adj[:0])
    return g


@pytest.mark.parametrize("o64", [False, True])
def test_validator_matches_oracle_on_planted_defects(ctx, o64):
    for c in csr_cases.cases():
        print(f"[validate] {c.name} o64={o64}", file=sys.stderr, flush=True)
        want = oracle.csr_validate(c.n, c.off, c.adj, c.sym)
        g = _dev_csr(ctx, c, o64)
        st, got = b.validate_csr(ctx, g, check_symmetric=c.sym)
        torch.cuda.synchronize()
        for k in ("failed", "rows_sorted", "symmetry_checked", "bad_entries", "first_bad_row"):
            assert got[k] == want[k], (c, k, got, want)
        assert (st == b.CC_OK) == (want["failed"] == 0), (c, st)
        ctx.sync_status()   # the validator clears the error word it set


def test_validator_reports_an_earlier_error_first(ctx):
    """A pending device error of an earlier call (here: the pair-list build's
    out-of-range id, which that kernel drops and flags) is returned before
    validating; the next call validates normally."""
    g = inputs.Graph(10, np.array([1, 2, 12], np.int32), np.array([2, 3, 4], np.int32))
    d = b.build_csr(ctx, g.n, g.u, g.v)
    torch.cuda.synchronize()
    with pytest.raises(b.CCError):
        b.validate_csr(ctx, d)
    st, r = b.validate_csr(ctx, d)
    assert st == b.CC_OK and r["failed"] == 0 and r["rows_sorted"] == 1


def test_validator_full_size_rmat_2_24(ctx):
    g = inputs.workload_rmat(24, 8, seed=2)
    dev = ctx.torch_device
    d = b.build_csr(ctx, g.n, torch.from_numpy(g.u).to(dev), torch.from_numpy(g.v).to(dev))
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    st, r = b.validate_csr(ctx, d)
    ev1.record()
    torch.cuda.synchronize()
    print(f"[validate] rmat24 m={d.m} {ev0.elapsed_time(ev1):.2f} ms", file=sys.stderr, flush=True)
    assert st == b.CC_OK
    assert {k: r[k] for k in ("failed", "rows_sorted", "symmetry_checked", "bad_entries", "first_bad_row")} == \
        {"failed": 0, "rows_sorted": 1, "symmetry_checked": 1, "bad_entries": 0, "first_bad_row": -1}
