"""Malformed and well-formed CSRs with planted defects, for the CSR
validator's tests.  Each case records what was planted (the defect bits,
the smallest defective row and the count of defective entries where the
definition fixes them); nothing here checks a CSR."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2008_03909_amd import inputs

OFFSET0, OFFSETN, MONOTONE, ID_RANGE, ASYMMETRIC = 1, 2, 4, 8, 16


class Case:
    def __init__(self, name, n, off, adj, bits, first=None, bad=None, sym=True, sorted_rows=None):
        self.name, self.n = name, int(n)
        self.off = np.asarray(off, np.int64)
        self.adj = np.asarray(adj, np.int32)
        self.bits, self.first, self.bad, self.sym = bits, first, bad, sym
        self.sorted_rows = sorted_rows

    def __repr__(self):
        return f"Case({self.name})"


def _csr(g, dedup=True):
    off, adj = oracle.csr_build(g.n, g.u, g.v, dedup)
    return np.asarray(off, np.int64).copy(), np.asarray(adj, np.int32).copy()


def _reverse_rows(off, adj):
    out = adj.copy()
    for v in range(len(off) - 1):
        out[off[v]:off[v + 1]] = adj[off[v]:off[v + 1]][::-1]
    return out


def _drop_entry(off, adj, v, w):
    """Removes one entry w from row v (the reverse entry stays)."""
    row = adj[off[v]:off[v + 1]]
    j = int(off[v] + np.flatnonzero(row == w)[0])
    adj2 = np.delete(adj, j)
    off2 = off.copy()
    off2[v + 1:] -= 1
    return off2, adj2


def cases():
    out = []
    g = inputs.rmat(10, 8 << 10, 0.57, 0.19, 0.19, seed=11)
    off, adj = _csr(g)
    n, m = g.n, len(adj)
    out.append(Case("valid-rmat", n, off, adj, 0, sorted_rows=1))
    out.append(Case("valid-unsorted", n, off, _reverse_rows(off, adj), 0, sorted_rows=0))
    gd = inputs.Graph(6, np.array([0, 0, 1, 2, 2, 4], np.int32), np.array([1, 1, 2, 3, 3, 4], np.int32), "dups")
    o2, a2 = _csr(gd, dedup=False)
    out.append(Case("valid-duplicates", gd.n, o2, a2, 0, sorted_rows=1))
    out.append(Case("empty", 5, np.zeros(6, np.int64), np.zeros(0, np.int32), 0, sorted_rows=1))

    r = int(np.flatnonzero(np.diff(off) > 0)[0])       # first non-empty row
    o = off.copy()
    o[0] = 1 if r == 0 else 0
    if r == 0:
        out.append(Case("offset0", n, o, adj, OFFSET0, first=0))
    o = off.copy()
    o[n] = m - 1                                             # an empty last row now runs backwards too
    out.append(Case("offsetN", n, o, adj, OFFSETN | (MONOTONE if o[n - 1] > m - 1 else 0), first=n - 1))
    v5 = int(np.flatnonzero(np.diff(off)[1:] > 0)[0]) + 1   # a row v5 >= 1 with entries
    o = off.copy()
    o[v5], o[v5 + 1] = off[v5 + 1], off[v5]                  # row v5 runs backwards
    out.append(Case("decreasing", n, o, adj, MONOTONE, first=v5))
    o = off.copy()
    o[10] = m + 7
    out.append(Case("beyond-m", n, o, adj, MONOTONE, first=9))
    o = off.copy()
    o[3] = -2
    out.append(Case("negative", n, o, adj, MONOTONE, first=2))
    a = adj.copy()
    jr = int(off[v5])
    a[jr] = n
    out.append(Case("id-high", n, off, a, ID_RANGE, first=v5, bad=1))
    a = adj.copy()
    a[-1] = -1
    a[0] = 2 ** 31 - 1
    out.append(Case("id-both-ends", n, off, a, ID_RANGE, first=r, bad=2))

    # asymmetric: drop (v, w) from row v; the entry (w, v) loses its reverse
    w = int(adj[off[v5]])
    if w == v5:
        w = int(adj[off[v5] + 1])
    o, a = _drop_entry(off, adj, v5, w)
    out.append(Case("asym-sorted", n, o, a, ASYMMETRIC, first=w, bad=1, sorted_rows=1))
    out.append(Case("asym-unsorted", n, o, _reverse_rows(o, a), ASYMMETRIC, sorted_rows=0))
    out.append(Case("asym-not-checked", n, o, a, 0, sym=False, sorted_rows=1))

    # a hub row far wider than a wave (walked by the whole wave)
    s = inputs.star(300, center=7)
    so, sa = _csr(s)
    out.append(Case("valid-star", s.n, so, sa, 0, sorted_rows=1))
    a = sa.copy()
    a[so[7] + 200] = -3
    out.append(Case("id-in-hub-row", s.n, so, a, ID_RANGE, first=7, bad=1))
    o, a = _drop_entry(so, sa, 123, 7)                       # leaf 123 forgets the hub
    out.append(Case("asym-hub", s.n, o, a, ASYMMETRIC, first=7, bad=1, sorted_rows=1))
    a = sa.copy()
    a[so[7]:so[8]] = sa[so[7]:so[8]][::-1]
    out.append(Case("unsorted-hub", s.n, so, a, 0, sorted_rows=0))

    # (0, 1) stored twice, (1, 0) once: symmetric as sets, not as multisets
    out.append(Case("dup-imbalance-sorted", 3, [0, 3, 4, 5], [1, 1, 2, 0, 0], 0, sorted_rows=1))
    out.append(Case("dup-imbalance-unsorted", 3, [0, 3, 4, 5], [1, 2, 1, 0, 0], ASYMMETRIC, sorted_rows=0))
    return out
