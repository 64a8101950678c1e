"""Benchmark: static connectivity throughput on one MI355X, plus incremental
updates/s with p50/p99 batch latency.

Default workload: R-MAT, n = 2^24, 8n tuples with (a,b,c,d) =
(0.57,0.19,0.19,0.05), seed 2, symmetrised and deduplicated on the device
(int32 CSR).  A step is one static connectivity call (init, k-out sampling,
IdentifyFrequent, compaction, finish, output) on the device-resident CSR with
the default variant (k-out k=2 hybrid + UF-Rem-CAS + SplitAtomicOne +
FindNaive).  edges/s = m / step time, m = directed edges after dedup.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def workload(name: str):
    from paper_2008_03909_amd import inputs

    if name == "rmat24":
        return inputs.workload_rmat(24, 8, seed=2), (
            "rmat n=2^24 edge_factor=8 (a,b,c,d)=(0.57,0.19,0.19,0.05) seed=2, symmetrized, deduplicated, int32 CSR")
    if name == "er16":
        return inputs.workload_er_2_16(), (
            "erdos-renyi n=2^16 pairs=2^19 seed=1, symmetrized, duplicates kept, int32 CSR")
    if name == "grid3d":
        return inputs.workload_grid3d(256, 0.35, seed=3), (
            "3d grid 256^3 bond percolation p=0.35 seed=3, symmetrized, int32 CSR")
    if name == "rmat27":
        return inputs.workload_rmat(27, 8, seed=4), (
            "rmat n=2^27 edge_factor=8 (a,b,c,d)=(0.57,0.19,0.19,0.05) seed=4, symmetrized, deduplicated, "
            "int64 offsets")
    raise SystemExit(f"unknown workload {name}")


def phase_alg_bytes(phase: str, n: int, m: int, o: int, n_nz: int, st: dict, k: int = 2, counts_in_init: bool = False,
                    na: int | None = None) -> float:
    """Algorithmic bytes of one launch of a phase of the default variant.

    n_nz = vertices with at least one edge; n_f / m_f = candidate vertices /
    their adjacency entries; every random 4-byte access counts 4 bytes.
    na = the vertices the per-vertex phases sweep (a renumbered CSR whose
    rows from na on are empty runs the algorithm on [0, na) only; n
    otherwise).  With k-out sampling the sampling kernel also clears the
    frequency counts, which the init then leaves alone (BFS and LDD leave
    them to the init; no sampling needs none)."""
    n_f, m_f, comps = st["candidates"], st["candidate_edges"], st["num_components"]
    na = n if na is None else na
    ca = comps - (n - na)                                # components among the swept vertices
    if phase == "init":
        return 4.0 * n + (4.0 * na if counts_in_init else 0.0)   # P (and count) writes
    if phase == "sample":
        return o * na + 4.0 * na + 16.0 * k * n_nz       # row bounds; count clear; k picks; k unions (2 reads + CAS)
    if phase == "mapback":
        return 8.0 * n + 8.0 * na + 4.0 * ca             # roots' original ids copied; P + non-roots' orig_of; new_of + labels
    if phase == "compress_count":
        return (4.0 + o) * na + 8.0 * n_nz               # P, degree; root read + count update
    if phase == "frequent":
        return 4.0 * na
    if phase == "compact":
        return (4.0 + o) * na + 4.0 * n_f
    if phase == "finish":
        return 2.0 * o * n_f + 12.0 * m_f                # row bounds; adjacency + 2 parent reads per edge
    if phase == "output":
        return 4.0 * na + 8.0 * (na - ca)                # P read; root read + write for non-roots
    return 0.0


CSRC = os.path.join(ROOT, "paper_2008_03909_amd", "csrc")


def kernel_digest(kernel: str):
    """Digest of a kernel's source: its definition (from the template line
    before ``__global__`` to the closing brace) plus the shared device
    header.  A profile taken from other source text is stale."""
    import glob
    import hashlib
    import re

    h = hashlib.sha256()
    found = False
    for path in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        text = open(path).read()
        m = re.search(r"__global__[^;{]*?\b" + re.escape(kernel) + r"\s*\(", text)
        if not m:
            continue
        a = text.rfind("\n\n", 0, m.start()) + 2
        depth, i = 0, text.index("{", m.end())
        for j in range(i, len(text)):
            depth += {"{": 1, "}": -1}.get(text[j], 0)
            if depth == 0:
                break
        h.update(text[a:j + 1].encode())
        found = True
        break
    if not found:
        return None
    h.update(open(os.path.join(CSRC, "cc_device.h"), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(kernel: str, workload_name: str):
    """HBM bytes per dispatch of `kernel` from a committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by the factor a plain
    copy kernel of known size gives), or None if there is none or it was
    taken from other kernel source."""
    path = os.path.join(ROOT, "profiles", f"pmc_{kernel}_{workload_name}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            a, b = line.split("=", 1)
            kv[a.strip()] = b.strip()
    if kv.get("kernel_digest") != kernel_digest(kernel):
        return None
    try:
        return float(kv["hbm_bytes_per_dispatch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(g, m: int, timed_labels=None, timed_ncomp=None):
    """The CPU oracle (sequential union-find over the pair list) on the same
    workload, one host core, median of 3 runs.  Its labels are also compared
    element by element with the labels of the timed GPU steps."""
    import numpy as np

    import oracle

    if not os.path.exists(oracle._SO):
        oracle.build()
    ts = []
    want = wc = None
    for _ in range(3):
        t = time.perf_counter()
        want, wc = oracle.uf_cc(g.n, g.u, g.v)
        ts.append(time.perf_counter() - t)
    match = None
    if timed_labels is not None:
        match = bool(np.array_equal(timed_labels, want)) and int(timed_ncomp) == int(wc)
    t = statistics.median(ts)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": m / t, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"full workload ({g.num_pairs} pairs), sequential union-find oracle, median of 3 runs "
                      f"({t:.2f} s each); host {cpu}, {os.cpu_count()} logical cpus",
            "labels_match_oracle": match}


def incremental(ctx, g, seed: int = 5, max_pairs: int | None = None, variant=None):
    """Insert the workload's pairs (shuffled) in batches of log-uniform size in
    [1e3, 1e7] interleaved with query batches of log-uniform size in
    [1e3, 1e6]; per-batch latency from HIP events on the issuing stream.
    The state is UF-Async with FindAtomicSplit unless another variant is
    given (the fastest UF-Async find here: 3.8e10 updates/s on RMAT 2^24
    against 2.5e10 for FindNaive and 2.8e10 for FindCompress)."""
    import numpy as np
    import torch

    from paper_2008_03909_amd import binding as b
    from paper_2008_03909_amd import inputs

    dev = ctx.torch_device
    su, sv = inputs.shuffle_pairs(g.u, g.v, seed)
    if max_pairs:
        su, sv = su[:max_pairs], sv[:max_pairs]
    du = torch.from_numpy(su).to(dev)
    dv = torch.from_numpy(sv).to(dev)
    qa, qb = inputs.query_pairs(g.n, 1_000_000, seed=6)
    dqa = torch.from_numpy(qa).to(dev)
    dqb = torch.from_numpy(qb).to(dev)
    qout = torch.empty(1_000_000, dtype=torch.uint8, device=dev)
    rng = np.random.default_rng(seed)
    v = variant if variant is not None else b.default_variant(finish=b.FIN_UF_ASYNC, find=b.FIND_ATOMIC_SPLIT)
    st = b.Stream(ctx, g.n, v)
    s = torch.cuda.current_stream()
    recs = []
    pos = 0
    total = du.numel()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while pos < total:
        if rng.random() < 0.5:
            k = min(inputs.log_uniform_int(1e3, 1e7, rng.random()), total - pos)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            st.insert(du[pos:pos + k], dv[pos:pos + k])
            e1.record(s)
            recs.append(("insert", k, e0, e1))
            pos += k
        else:
            q = inputs.log_uniform_int(1e3, 1e6, rng.random())
            off = int(rng.integers(0, 1_000_000 - q + 1))
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            st.query(dqa[off:off + q], dqb[off:off + q], out=qout[:q])
            e1.record(s)
            recs.append(("query", q, e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st.sync_status()
    st.close()
    ins = [(k, a.elapsed_time(bb)) for kind, k, a, bb in recs if kind == "insert"]
    qs = [(k, a.elapsed_time(bb)) for kind, k, a, bb in recs if kind == "query"]
    lat = sorted(ms for _, ms in ins + qs)

    def pct(xs, p):
        xs = sorted(xs)
        return xs[min(len(xs) - 1, int(round(p / 100.0 * (len(xs) - 1))))] if xs else None

    ins_ms = sum(ms for _, ms in ins)
    q_ms = sum(ms for _, ms in qs)
    return {
        "updates_per_s": sum(k for k, _ in ins) / (ins_ms / 1e3) if ins_ms else None,
        "queries_per_s": sum(k for k, _ in qs) / (q_ms / 1e3) if q_ms else None,
        "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
        "insert_p50_ms": pct([ms for _, ms in ins], 50), "insert_p99_ms": pct([ms for _, ms in ins], 99),
        "query_p50_ms": pct([ms for _, ms in qs], 50), "query_p99_ms": pct([ms for _, ms in qs], 99),
        "batches": len(recs), "inserted_pairs": sum(k for k, _ in ins), "queried_pairs": sum(k for k, _ in qs),
        "wall_s": wall,
        "finish": v.name().split("+")[-1],
        "note": "undirected pair inserts (duplicates and self-loops included as no-op inserts); latency is "
                "device time per batch from HIP events; batches run back to back on one stream",
    }


def mixed(ctx, g, seed: int = 7, total_ops: int = 20_000_000):
    """Mixed batches (cc_process_batch): the workload's pairs, shuffled, as
    inserts, interleaved 50/50 with uniform random queries, in batches of
    log-uniform size in [1e3, 1e7] operations; device time per batch.  One
    type-1 stream (inserts and queries in one kernel) and one type-3 stream
    (Rem-CAS with SpliceAtomic: inserts, then queries)."""
    import numpy as np
    import torch

    from paper_2008_03909_amd import binding as b
    from paper_2008_03909_amd import inputs

    dev = ctx.torch_device
    rng = np.random.default_rng(seed)
    su, sv = inputs.shuffle_pairs(g.u, g.v, seed)
    half = min(total_ops // 2, su.shape[0])
    qa, qb = inputs.query_pairs(g.n, half, seed=seed + 1)
    kind = np.concatenate([np.zeros(half, np.uint8), np.ones(half, np.uint8)])
    u = np.concatenate([su[:half], qa])
    w = np.concatenate([sv[:half], qb])
    perm = rng.permutation(2 * half)
    dk = torch.from_numpy(kind[perm]).to(dev)
    du = torch.from_numpy(u[perm]).to(dev)
    dw = torch.from_numpy(w[perm]).to(dev)
    out = torch.empty(2 * half, dtype=torch.uint8, device=dev)
    sizes = []
    pos = 0
    while pos < 2 * half:
        k = min(inputs.log_uniform_int(1e3, 1e7, rng.random()), 2 * half - pos)
        sizes.append((pos, k))
        pos += k
    res = {}
    for name, v in (("type1_uf_async", b.default_variant(finish=b.FIN_UF_ASYNC, find=b.FIND_NAIVE)),
                    ("type3_rem_splice", b.default_variant(splice=b.SPLICE_ATOMIC))):
        st = b.Stream(ctx, g.n, v)
        s = torch.cuda.current_stream()
        recs = []
        torch.cuda.synchronize()
        for p0, k in sizes:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            st.process(dk[p0:p0 + k], du[p0:p0 + k], dw[p0:p0 + k], out=out[p0:p0 + k])
            e1.record(s)
            recs.append((k, e0, e1))
        torch.cuda.synchronize()
        st.sync_status()
        st.close()
        ms = sorted(a.elapsed_time(bb) for _, a, bb in recs)
        tot = sum(ms)
        res[name] = {"ops_per_s": 2 * half / (tot / 1e3), "p50_ms": ms[len(ms) // 2],
                     "p99_ms": ms[min(len(ms) - 1, int(round(0.99 * (len(ms) - 1))))], "batches": len(ms)}
    res["ops"] = 2 * half
    res["note"] = "half inserts (workload pairs), half uniform queries, shuffled together; device time per batch"
    return res


def serving(ctx, g, capacity_pairs_per_s: float | None = None, loads=(0.0, 0.3, 0.6, 0.9, 1.2), requests: int = 300,
            seed: int = 5, variant=None):
    """Poisson arrivals through the serving loop (continuous batching): insert
    requests of log-uniform size in [1e3, 1e7] pairs (the workload's pairs,
    shuffled) and query requests in [1e3, 1e6] random pairs, 50/50, at an
    offered load given as a fraction of a capacity (pairs/s).  Payloads live
    in pinned host memory, which the kernels read (and answer into) in place
    over PCIe, inside the measured latency.  Load
    0.0 means every request arrives at once (closed loop); its throughput is
    the capacity the other loads are scaled to."""
    import numpy as np

    from paper_2008_03909_amd import binding as b
    from paper_2008_03909_amd import inputs

    su, sv = inputs.shuffle_pairs(g.u, g.v, seed)
    # warm-up: the first launches of the server's kernels load their code,
    # which must not land in the closed-loop capacity run
    wa = np.ascontiguousarray(su[:1000]).astype(np.int32)
    wb = np.ascontiguousarray(sv[:1000]).astype(np.int32)
    wsrv = b.Server(ctx, g.n, variant=variant, budget_bytes=1 << 20, num_streams=2, max_inflight=4)
    wsrv.run_trace(np.array([0, 1]), np.zeros(2), np.array([0, 0]), np.array([1000, 1000]), wa, wb)
    wsrv.close()
    res = []
    for li, load in enumerate(loads):
        rng = np.random.default_rng(seed + li)
        types, starts, lens, A, B = [], [], [], [], []
        pe, pos = 0, 0
        for i in range(requests):
            t = int(rng.random() < 0.5)
            if t == 0 and pe < su.size:
                k = min(inputs.log_uniform_int(1e3, 1e7, rng.random()), su.size - pe)
                A.append(su[pe:pe + k])
                B.append(sv[pe:pe + k])
                pe += k
            else:
                t = 1
                k = inputs.log_uniform_int(1e3, 1e6, rng.random())
                qa, qb = inputs.query_pairs(g.n, k, seed=seed * 7919 + 31 * li + i)
                A.append(qa)
                B.append(qb)
            types.append(t)
            starts.append(pos)
            lens.append(k)
            pos += k
        lens_a = np.array(lens, np.float64)
        if load <= 0.0:
            arrivals = np.zeros(len(types))
        else:
            rate = load * capacity_pairs_per_s / lens_a.mean()      # requests per second
            arrivals = np.cumsum(rng.exponential(1.0 / rate, len(types)))
        # request payloads and answers in pinned host memory (read and written in place by the kernels)
        import torch
        pa = torch.from_numpy(np.concatenate(A).astype(np.int32)).pin_memory()
        pb = torch.from_numpy(np.concatenate(B).astype(np.int32)).pin_memory()
        po = torch.zeros(pa.numel(), dtype=torch.uint8).pin_memory()
        srv = b.Server(ctx, g.n, variant=variant, budget_bytes=2 << 30, num_streams=2, max_inflight=64)
        mode = "stamped" if srv.stamped else "barrier"
        t0 = time.perf_counter()
        _, lat = srv.run_trace(np.array(types), arrivals, np.array(starts), np.array(lens),
                               pa.numpy(), pb.numpy(), po.numpy())
        wall = time.perf_counter() - t0
        srv.close()
        ty = np.array(types)
        ins_pairs = float(lens_a[ty == 0].sum())
        if load <= 0.0:
            capacity_pairs_per_s = float(lens_a.sum()) / wall
        res.append({
            "mode": mode, "offered_load": load, "requests": len(types), "inserted_pairs": int(ins_pairs),
            "queried_pairs": int(lens_a[ty == 1].sum()), "wall_s": round(wall, 4),
            "updates_per_s": ins_pairs / wall, "pairs_per_s": float(lens_a.sum()) / wall,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "insert_p50_ms": float(np.percentile(lat[ty == 0], 50) * 1e3) if np.any(ty == 0) else None,
            "query_p50_ms": float(np.percentile(lat[ty == 1], 50) * 1e3) if np.any(ty == 1) else None,
            "insert_p99_ms": float(np.percentile(lat[ty == 0], 99) * 1e3) if np.any(ty == 0) else None,
            "query_p99_ms": float(np.percentile(lat[ty == 1], 99) * 1e3) if np.any(ty == 1) else None,
        })
    return res


def _time_ms(fn, reps: int = 10) -> float:
    import torch

    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def calibration(ctx, csr, n: int, m: int, o: int):
    """Roofline anchors on the same device: a 1 GiB stream copy, and the
    paper's MapEdges / GatherEdges primitives on the workload's CSR."""
    import torch

    from paper_2008_03909_amd import binding as b

    dev = ctx.torch_device
    nb = 1 << 30
    src = torch.empty(nb, dtype=torch.uint8, device=dev)
    dst = torch.empty(nb, dtype=torch.uint8, device=dev)
    t_copy = _time_ms(lambda: b.calib_copy(src, dst))
    del src, dst
    vals = torch.arange(n, dtype=torch.int32, device=dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    t_map = _time_ms(lambda: b.calib_edges(csr, None, out))
    t_gather = _time_ms(lambda: b.calib_edges(csr, vals, out))
    map_bytes = (o + 4) * n + 4 * m
    gather_bytes = (o + 4) * n + 8 * m
    return {
        "copy_gbs": round(2 * nb / (t_copy / 1e3) / 1e9, 1),
        "map_edges_ms": round(t_map, 4), "map_edges_gbs": round(map_bytes / (t_map / 1e3) / 1e9, 1),
        "gather_edges_ms": round(t_gather, 4), "gather_edges_gbs": round(gather_bytes / (t_gather / 1e3) / 1e9, 1),
        "gather_edges_edges_per_s": m / (t_gather / 1e3),
    }


def sweep(ctx, csr, g, workload_name: str, reps: int = 5, check: bool = True, rcsr=None):
    """Time every sampling x finish variant (median of `reps` after one warm-up)
    and check every labelling against the CPU oracle.  Extra rows vary the
    k-out edge choice and k under the default finish.  With rcsr (a
    renumbered CSR of the same graph) the calls are the mapped ones, on the
    layout the static call of the benchmark uses."""
    import numpy as np
    import torch

    import oracle
    from paper_2008_03909_amd import binding as b

    want = None
    if check:
        if not os.path.exists(oracle._SO):
            oracle.build()
        want, _ = oracle.uf_cc(g.n, g.u, g.v)
    vs = b.all_variants(extended=True)
    base = b.default_variant()
    extra = [base.copy(kout_mode=b.KOUT_AFFOREST), base.copy(kout_mode=b.KOUT_PURE),
             base.copy(kout_k=1), base.copy(kout_k=3), base.copy(kout_mode=b.KOUT_AFFOREST, kout_k=1),
             base.copy(kout_mode=b.KOUT_MAXDEG)]
    rows = []
    dev = ctx.torch_device
    labels = torch.empty(csr.n, dtype=torch.int32, device=dev)
    ncomp = torch.empty(1, dtype=torch.int64, device=dev)
    def call(v):
        if rcsr is not None:
            b.connectivity_csr_mapped(ctx, rcsr, v, labels=labels, ncomp=ncomp)
        else:
            b.connectivity_csr(ctx, csr, v, labels=labels, ncomp=ncomp)

    for i, v in enumerate(vs + extra):
        call(v)
        torch.cuda.synchronize()
        ok = True
        if want is not None:
            ok = bool(np.array_equal(labels.cpu().numpy(), want))
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            call(v)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        st = ctx.last_stats()
        ms = statistics.median(ts)
        rows.append({"variant": v.name(), "index": i if i < len(vs) else None, "ms": round(ms, 4),
                     "edges_per_s": csr.m / (ms / 1e3), "labels_match_oracle": ok,
                     "sample_rounds": st["sample_rounds"], "finish_rounds": st["finish_rounds"],
                     "candidates": st["candidates"], "candidate_edges": st["candidate_edges"],
                     "lmax_size": st["lmax_size"]})
        log(f"  [{i:2d}] {v.name():40s} {ms:9.3f} ms  match={ok} rounds={st['sample_rounds']}/{st['finish_rounds']}")
    ctx.sync_status()
    return rows


def amsf_leg(ctx, csr, n: int, m: int, ms_conn: float, steps: int, rcsr=None) -> dict:
    """Approximate MSF (Section 5.1) with exponential weights of mean 1 (the
    paper's weighting, a function of the pair of original vertices), eps =
    0.25, on the layout of the static call (the renumbered CSR rcsr when
    given).  Timed outside the main region; per-phase times from the call's
    own events."""
    import numpy as np
    import torch

    from paper_2008_03909_amd import binding as b
    from paper_2008_03909_amd import inputs

    t = time.perf_counter()
    g = rcsr if rcsr is not None else csr
    off_h = g.offsets.cpu().numpy()
    adj_h = g.adj.cpu().numpy()
    rows = np.repeat(np.arange(n, dtype=np.int32), np.diff(off_h))
    if rcsr is not None:
        orig = rcsr.orig_of.cpu().numpy()
        rows, adj_h = orig[rows], orig[adj_h]
    w = inputs.pair_weights(n, rows, adj_h, seed=77, mean=1.0)
    del rows, adj_h, off_h
    wt = torch.from_numpy(w).to(ctx.torch_device)
    del w
    log(f"amsf weights in {time.perf_counter() - t:.1f}s")
    opt = b.amsf_options()
    if rcsr is not None:
        def call():
            return b.amsf_csr_mapped(ctx, rcsr, wt, opt)
    else:
        def call():
            return b.amsf_csr(ctx, csr, wt, opt)
    for _ in range(2):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, _, _, _, ne, tw = call()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # phase breakdown from a separate pass (phase events slow the calls down)
    ctx.set_timing(True)
    ctx.phase_times_reset()
    for _ in range(steps):
        call()
    torch.cuda.synchronize()
    ctx.set_timing(False)
    ph = {k: round(v[0] / steps, 4) for k, v in ctx.phase_times().items()}
    st = ctx.last_stats()
    res = {"ms": ms, "edges_per_s": m / (ms / 1e3), "epsilon": float(opt.epsilon),
           "light_fraction": float(opt.light_fraction), "forest_edges": int(ne.item()),
           "weight": float(tw.item()), "light_buckets": st["sample_rounds"], "rounds": st["finish_rounds"],
           "vs_connectivity": ms / ms_conn, "phase_ms_per_call": ph}
    log(f"amsf: {ms:.3f} ms ({ms / ms_conn:.2f}x connectivity), {res['forest_edges']} edges, "
        f"light buckets {res['light_buckets']}, rounds {res['rounds']}, phases {ph}")
    del wt
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24", choices=["rmat24", "er16", "grid3d", "rmat27"])
    ap.add_argument("--variant", default="default", help="'default' or an index into the 80-variant list")
    ap.add_argument("--layout", default="auto", choices=["auto", "given", "degree"],
                    help="CSR of the timed static call: as given, or renumbered by decreasing degree at ingest "
                         "(labels mapped back inside the call); auto = degree on the R-MAT workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-incremental", action="store_true")
    ap.add_argument("--no-forest", action="store_true", help="skip the spanning-forest timing")
    ap.add_argument("--no-amsf", action="store_true", help="skip the approximate-MSF timing")
    ap.add_argument("--phases", action="store_true", help="print per-phase times to stderr")
    ap.add_argument("--sweep", default="", help="also time every variant (80 main + 36 further finishes + k-out "
                                                 "edge choices); write the rows to this JSON file")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding the graph over several GPUs "
              f"is designed but not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2008_03909_amd import binding as b

    assert torch.cuda.is_available(), "no GPU"
    t = time.perf_counter()
    g, desc = workload(args.workload)
    log(f"generated {g} in {time.perf_counter() - t:.1f}s")

    ctx = b.Context(0)
    dev = ctx.torch_device
    du = torch.from_numpy(g.u).to(dev)
    dv = torch.from_numpy(g.v).to(dev)
    dedup = args.workload != "er16"
    o64 = args.workload == "rmat27"
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    csr = b.build_csr(ctx, g.n, du, dv, dedup=dedup, offsets_64bit=o64)
    e1.record()
    torch.cuda.synchronize()
    ingest_ms = e0.elapsed_time(e1)
    # the timed static call runs on the layout chosen for the workload: on the
    # power-law graphs a CSR renumbered by decreasing degree at ingest
    # (labels mapped back to the original numbering inside the timed call)
    layout = args.layout if args.layout != "auto" else ("degree" if args.workload in ("rmat24", "rmat27") else "given")
    rcsr = None
    relabel_ms = None
    if layout == "degree":
        torch.cuda.synchronize()
        e0.record()
        rcsr = b.build_csr_degree_order(ctx, g.n, du, dv, dedup=dedup, offsets_64bit=o64)
        e1.record()
        torch.cuda.synchronize()
        relabel_ms = e0.elapsed_time(e1)
        assert rcsr.m == csr.m
    del du, dv
    n, m = csr.n, csr.m
    o = 8 if o64 else 4
    deg = (csr.offsets[1:] - csr.offsets[:-1])
    n_nz = int((deg > 0).sum().item())
    del deg
    log(f"device CSR: n={n} m={m} nonisolated={n_nz} ingest {ingest_ms:.1f} ms")

    if args.variant == "default":
        v = b.default_variant()
    else:
        v = b.all_variants()[int(args.variant)]
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    ncomp = torch.empty(1, dtype=torch.int64, device=dev)
    ws = ctx.workspace(b.workspace_bytes(n, m, v))
    if rcsr is not None:
        def static_call():
            b.connectivity_csr_mapped(ctx, rcsr, v, labels=labels, ncomp=ncomp)
    else:
        def static_call():
            b.connectivity_csr(ctx, csr, v, labels=labels, ncomp=ncomp)
    # warm-up: one cold call, then the rest with every phase timed, which
    # names the dominant phase
    static_call()
    torch.cuda.synchronize()
    ctx.set_timing(True)
    ctx.phase_times_reset()
    for _ in range(max(args.warmup - 1, 1)):
        static_call()
    torch.cuda.synchronize()
    ctx.set_timing(False)
    ctx.sync_status()
    warm = ctx.phase_times()
    dom = max(warm, key=lambda k_: warm[k_][0] / max(warm[k_][1], 1)) if warm else "sample"

    # timed region: K steps; HIP events on the call's stream around the
    # dominant phase only (each recorded event makes the stream drain the
    # work before it, so timing every phase would slow the steps down)
    ctx.set_timing(True, only=dom)
    ctx.phase_times_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        static_call()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.set_timing(False)
    ctx.sync_status()
    timed = ctx.phase_times()
    st = ctx.last_stats()
    timed_labels = labels.cpu().numpy()      # the last timed step's output, checked by the CPU leg
    timed_ncomp = int(ncomp.item())
    # per-phase breakdown from a separate pass with every phase timed; the
    # dominant phase keeps the timed region's own measurement
    ctx.set_timing(True)
    ctx.phase_times_reset()
    for _ in range(args.steps):
        static_call()
    torch.cuda.synchronize()
    ctx.set_timing(False)
    phases = ctx.phase_times()
    if dom in timed:
        phases[dom] = timed[dom]
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = m / (ms_step / 1e3)
    log(f"static: {ms_step:.3f} ms/step, {value:.3e} edges/s, components={st['num_components']}")

    alg_total = 0.0
    ph_out = {}
    for name, (ms, cnt) in phases.items():
        avg = ms / max(cnt, 1)
        ab = phase_alg_bytes(name, n, m, o, n_nz, st, k=v.kout_k,
                             counts_in_init=v.sample in (b.SAMPLE_BFS, b.SAMPLE_LDD),
                             na=rcsr.n_active if rcsr is not None else n)
        alg_total += ab * cnt / args.steps
        ph_out[name] = {"avg_ms": round(avg, 4), "launches": cnt, "alg_bytes": ab,
                        "alg_gbs": round(ab / (avg / 1e3) / 1e9, 1) if avg > 0 else None}
    if args.phases:
        for k_, x in ph_out.items():
            log(f"  {k_:16s} {x}")
    sampler_kernel = {b.SAMPLE_KOUT: "k_kout", b.SAMPLE_BFS: "bfs levels (k_bfs_*)",
                      b.SAMPLE_LDD: "ldd rounds (k_ldd_wake, k_expand*)"}.get(v.sample, "none")
    dom_kernel = {"sample": sampler_kernel, "compress_count": "k_compress_count", "init": "k_init",
                  "frequent": "k_argmax", "compact": "k_compact", "finish": "k_fin", "output": "k_output"}.get(dom, dom)
    achieved = ph_out[dom]["alg_gbs"]
    traffic = read_traffic(dom_kernel, args.workload)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4) if achieved else None,
                "traffic": traffic, "kernel": dom_kernel, "phase": dom,
                "alg_bytes_per_launch": ph_out[dom]["alg_bytes"], "avg_launch_ms": ph_out[dom]["avg_ms"]}
    if traffic:
        # the measured HBM bytes per launch over this run's launch time: the
        # rate the memory system actually delivered (line-granular traffic)
        tg = traffic / (ph_out[dom]["avg_ms"] / 1e3) / 1e9
        roofline["traffic_gbs"] = round(tg, 1)
        roofline["traffic_frac"] = round(tg / HBM_PEAK_GBS, 4)

    out = {
        "metric": "static CC edges/s + HBM GB/s; incremental updates/s with p50/p99 latency",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "m": m, "nonisolated": n_nz, "variant": v.name(),
                   "num_components": st["num_components"], "parallelism": "single-gpu",
                   "layout": ("CSR renumbered by decreasing degree at ingest; the algorithm runs on the "
                              f"{rcsr.n_active} vertices with edges (the isolated ones come last); labels of all "
                              "vertices mapped back to the original numbering inside the timed call"
                              if rcsr is not None else "CSR as built")},
        "hbm_gbs_alg": round(alg_total / (ms_step / 1e3) / 1e9, 1),
        "roofline": roofline,
        "phases": ph_out,
        "stats": st,
        "ingest": {"ms": ingest_ms, "pairs": g.num_pairs, "pairs_per_s": g.num_pairs / (ingest_ms / 1e3),
                   "degree_order_ms": relabel_ms},
    }
    del ws
    forest_ok = v.finish == b.FIN_UF_ASYNC or (v.finish == b.FIN_UF_REM_CAS and v.splice != b.SPLICE_ATOMIC)
    if not args.no_forest and forest_ok:
        # spanning forest with the default variant on the layout the static
        # call used (outside the timed region above); on a renumbered CSR its
        # edges and labels come back in the original numbering
        if rcsr is not None:
            def forest_call():
                return b.spanning_forest_csr_mapped(ctx, rcsr, v)
        else:
            def forest_call():
                return b.spanning_forest_csr(ctx, csr, v)
        for _ in range(2):
            forest_call()
        torch.cuda.synchronize()
        t0f = time.perf_counter()
        for _ in range(args.steps):
            _, _, _, ne = forest_call()
        torch.cuda.synchronize()
        ms_f = (time.perf_counter() - t0f) * 1e3 / args.steps
        out["spanning_forest"] = {"ms": ms_f, "edges_per_s": m / (ms_f / 1e3),
                                  "forest_edges": int(ne.item()), "vs_connectivity": ms_f / ms_step,
                                  "layout": layout}
        log(f"spanning forest: {ms_f:.3f} ms ({ms_f / ms_step:.2f}x connectivity), {int(ne.item())} edges")
    if not args.no_amsf:
        out["amsf"] = amsf_leg(ctx, csr, n, m, ms_step, args.steps, rcsr=rcsr)
        out["amsf"]["layout"] = layout
    if args.sweep:
        log("variant sweep ...")
        rows = sweep(ctx, csr, g, args.workload, rcsr=rcsr)
        with open(args.sweep, "w") as f:
            json.dump({"workload": desc, "n": n, "m": m, "rows": rows}, f, indent=1)
        best = min(rows[:80], key=lambda r: r["ms"])
        best_all = min(rows, key=lambda r: r["ms"])
        out["sweep"] = {"variants": len(rows), "all_match_oracle": all(r["labels_match_oracle"] for r in rows),
                        "best": best["variant"], "best_ms": best["ms"], "best_edges_per_s": best["edges_per_s"],
                        "best_any_row": best_all["variant"], "best_any_row_ms": best_all["ms"],
                        "file": os.path.basename(args.sweep), "layout": layout}
    del rcsr
    out["calibration"] = calibration(ctx, csr, n, m, o)
    log(f"calibration: {out['calibration']}")
    if not args.no_incremental:
        log("incremental stream ...")
        out["incremental"] = incremental(ctx, g)
        log("mixed batches ...")
        out["mixed_batches"] = mixed(ctx, g)
        log(f"mixed: {out['mixed_batches']}")
        log(f"incremental: {out['incremental']['updates_per_s']:.3e} updates/s, "
            f"p50 {out['incremental']['p50_ms']:.3f} ms, p99 {out['incremental']['p99_ms']:.3f} ms")
        log("serving loop (Poisson arrivals) ...")
        out["serving"] = serving(ctx, g)
        # the same traces with the barrier between insert and query phases
        # (Rem-CAS / SplitAtomicOne, whose splices rewrite links)
        out["serving_barrier_mode"] = serving(ctx, g, loads=(0.0, 0.9), variant=b.default_variant(
            finish=b.FIN_UF_REM_CAS, splice=b.SPLICE_SPLIT_ONE, find=b.FIND_NAIVE))
        for r in out["serving"] + out["serving_barrier_mode"]:
            log(f"serving {r['mode']} load {r['offered_load']}: {r['pairs_per_s']:.3e} pairs/s, "
                f"p50 {r['p50_ms']:.3f} ms, p99 {r['p99_ms']:.3f} ms")
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(g, m, timed_labels, timed_ncomp)
        out["labels_match_oracle"] = out["cpu_baseline"]["labels_match_oracle"]
        log(f"cpu baseline: {out['cpu_baseline']['value']:.3e} edges/s, "
            f"timed labels match the oracle: {out['labels_match_oracle']}")
    out["host"] = platform.node()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
