"""Host-side accounting of bench.py: the algorithmic bytes per phase (the
roofline's numerator) and the per-vertex terms of a call restricted to the
vertices with edges."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402

ST = {"candidates": 1000, "candidate_edges": 5000, "num_components": 900}


def test_sweeping_every_vertex_is_the_default():
    for ph in ("init", "sample", "mapback", "compress_count", "frequent", "compact", "finish", "output"):
        assert bench.phase_alg_bytes(ph, 10_000, 80_000, 4, 9_000, ST) == \
            bench.phase_alg_bytes(ph, 10_000, 80_000, 4, 9_000, ST, na=10_000)


def test_restricted_call_counts_only_the_swept_vertices():
    n, na, o, nnz = 10_000, 6_000, 4, 6_000
    # the 4,000 vertices after na are components of their own
    st = dict(ST, num_components=4_000 + 300)
    full = {ph: bench.phase_alg_bytes(ph, n, 80_000, o, nnz, st) for ph in ("sample", "compress_count", "frequent")}
    part = {ph: bench.phase_alg_bytes(ph, n, 80_000, o, nnz, st, na=na) for ph in full}
    assert full["sample"] - part["sample"] == (o + 4) * (n - na)
    assert full["compress_count"] - part["compress_count"] == (4 + o) * (n - na)
    assert full["frequent"] - part["frequent"] == 4 * (n - na)
    # the init still writes every parent; the gather still writes every label
    assert bench.phase_alg_bytes("init", n, 80_000, o, nnz, st, na=na) == 4 * n
    assert bench.phase_alg_bytes("mapback", n, 80_000, o, nnz, st, na=na) == 8 * n + 8 * na + 4 * 300
    # output: every swept vertex read, non-roots among them read and written
    assert bench.phase_alg_bytes("output", n, 80_000, o, nnz, st, na=na) == 4 * na + 8 * (na - 300)
