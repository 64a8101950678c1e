"""Learned variant selector: corpus, training and evaluation drivers.

The model and its kernels live in the HIP library (features, BF16 MLP
forward / backward / Adam); this module only prepares inputs and drives the
library.  The selector changes speed, never labels.

Corpus: synthetic graphs whose family and size follow from a seed -- ER
(average degree log-uniform in [1, 64]), R-MAT (a in [0.45, 0.70], d = 0.05,
b = c, edge factor 8), percolated 2D grids (p in [0.45, 1]) and 3D grids
(p in [0.2, 1]), stars, chains in random id order, and disjoint unions of
2-8 of these; n log-uniform in [2^lo, 2^hi].  Graphs with seed % 10 == 0
are held out.  Each graph records its 16 features (degree statistics,
sampled first-neighbour statistics, a budgeted BFS probe; computed on the
device) and the time of every arm (median of up to 3 runs; arms that reach
the round limit are censored at their elapsed time).  Targets are
log(t_arm) - log(min_arm t).
"""
from __future__ import annotations

import concurrent.futures as cf
import math
import statistics
import sys
import time

import numpy as np
import torch

from . import binding as b
from . import inputs

FAMILIES = ("er", "rmat", "grid2d", "grid3d", "star", "chain", "union")


def arms():
    """The K = 24 arms: {none, k-out, BFS, LDD} x {Rem-CAS/SplitAtomicOne,
    Rem-CAS/SpliceAtomic, Async/FindAtomicSplit, Shiloach-Vishkin}, then four
    k-out edge choices with Rem-CAS/SplitAtomicOne: hybrid k = 1, afforest
    k = 1 and k = 2, hybrid k = 3; then k-out with the further finishes
    UF-Early/FindNaive, UF-Hooks/FindAtomicSplit and label propagation, and
    the max-degree edge choice with Rem-CAS/SplitAtomicOne."""
    base = b.default_variant()
    fins = [dict(finish=b.FIN_UF_REM_CAS, splice=b.SPLICE_SPLIT_ONE, find=b.FIND_NAIVE),
            dict(finish=b.FIN_UF_REM_CAS, splice=b.SPLICE_ATOMIC, find=b.FIND_NAIVE),
            dict(finish=b.FIN_UF_ASYNC, splice=0, find=b.FIND_ATOMIC_SPLIT),
            dict(finish=b.FIN_SV, splice=0, find=0)]
    out = []
    for s in (b.SAMPLE_NONE, b.SAMPLE_KOUT, b.SAMPLE_BFS, b.SAMPLE_LDD):
        for f in fins:
            out.append(base.copy(sample=s, **f))
    for k, mode in ((1, b.KOUT_HYBRID), (1, b.KOUT_AFFOREST), (2, b.KOUT_AFFOREST), (3, b.KOUT_HYBRID)):
        out.append(base.copy(kout_k=k, kout_mode=mode))
    out.append(base.copy(finish=b.FIN_UF_EARLY, find=b.FIND_NAIVE, splice=0))
    out.append(base.copy(finish=b.FIN_UF_HOOKS, find=b.FIND_ATOMIC_SPLIT, splice=0))
    out.append(base.copy(finish=b.FIN_LP, find=0, splice=0))
    out.append(base.copy(kout_mode=b.KOUT_MAXDEG))
    return out


# End-to-end cost of the features, the forward pass and the host's wait for
# the choice, measured on held-out graphs as the selector's time minus its
# chosen arm's time (about 27 us); used to decide where the model pays.
SELECTOR_OVERHEAD_MS = 0.027
GATE_CANDIDATES = (0, 1 << 12, 1 << 13, 1 << 14, 1 << 15, 1 << 16, 1 << 17, 1 << 18)


def choose_gate(times, n, picks, overhead_ms=SELECTOR_OVERHEAD_MS):
    """The small-graph gate (min_vertices, arm) that minimises the mean time
    over training graphs when graphs below min_vertices run one fixed arm
    (no selector cost) and the rest run the model's pick plus its overhead.
    min_vertices = 0 means no gate."""
    times = np.asarray(times, np.float64)
    n = np.asarray(n)
    rows = np.arange(times.shape[0])
    model_cost = times[rows, picks] + overhead_ms
    best = (float(model_cost.mean()), 0, -1)
    for th in GATE_CANDIDATES[1:]:
        below = n < th
        if not below.any():
            continue
        arm = int(np.argmin(times[below].mean(0)))
        cost = float(np.where(below, times[:, arm], model_cost).mean())
        if cost < best[0]:
            best = (cost, int(th), arm)
    return best[1], best[2]


# Output bias given to a pruned arm: far above any predicted log-time
# ratio, so the decision's argmin never lands on it (BF16 holds it as 9984).
PRUNED_BIAS = 1.0e4


def prune_arms(pred, times, clip=20.0):
    """Backward elimination of arms on training rows: repeatedly drop the arm
    whose removal most lowers the mean time of the model's pick (argmin of
    pred over the arms kept), while some removal lowers it.  An arm that the
    model over-rates (picked where it is rarely good) goes; an arm it picks
    well stays.  Times are clipped at clip x the row's median so that one
    disturbed measurement cannot decide.  Returns the boolean keep mask."""
    pred = np.asarray(pred, np.float64)
    T = np.asarray(times, np.float64)
    T = np.minimum(T, clip * np.median(T, axis=1, keepdims=True))
    rows = np.arange(T.shape[0])

    def cost(keep):
        return T[rows, np.where(keep[None, :], pred, np.inf).argmin(1)].mean()

    keep = np.ones(T.shape[1], bool)
    cur = cost(keep)
    while keep.sum() > 2:
        trials = []
        for a in np.flatnonzero(keep):
            k2 = keep.copy()
            k2[a] = False
            trials.append((cost(k2), a))
        c, a = min(trials)
        if c >= cur * (1.0 - 1e-4):
            break
        keep[a] = False
        cur = c
    return keep


def apply_pruning(master, K, keep):
    """Sets the output bias of every arm not kept to PRUNED_BIAS (the last K
    entries of the FP32 master parameters are the output biases)."""
    m = np.array(master, np.float32, copy=True)
    m[len(m) - K:][~np.asarray(keep, bool)] = PRUNED_BIAS
    return m


def default_arm_index() -> int:
    return 4   # k-out + Rem-CAS/SplitAtomicOne/FindNaive: the paper's default


def decision_tree_arm(features) -> int:
    """The paper's text rules (its decision-tree figure is missing): no
    sampling when m/n < 3, otherwise k-out; finish with UF-Rem-CAS."""
    return 0 if features[14] > 0.5 else 4


def _member(rng, n):
    fam = int(rng.integers(0, 6))
    return _family_graph(fam, n, rng)


def _family_graph(fam, n, rng):
    seed = int(rng.integers(0, 2**31))
    n = max(int(n), 16)
    if fam == 0:
        deg = math.exp(rng.uniform(0, math.log(64)))
        return inputs.er(n, max(1, int(deg * n / 2)), seed)
    if fam == 1:
        a = rng.uniform(0.45, 0.70)
        bc = (1 - a - 0.05) / 2
        scale = max(4, int(round(math.log2(n))))
        return inputs.rmat(scale, 8 << scale, a, bc, bc, seed)
    if fam == 2:
        side = max(2, int(round(math.sqrt(n))))
        return inputs.grid(2, side, rng.uniform(0.45, 1.0), seed)
    if fam == 3:
        side = max(2, int(round(n ** (1 / 3))))
        return inputs.grid(3, side, rng.uniform(0.2, 1.0), seed)
    if fam == 4:
        return inputs.star(n, int(rng.integers(0, n)))
    return inputs.chain(n, seed)


def corpus_graph(seed: int, lo: int = 12, hi: int = 22):
    """The corpus graph of a seed: (family name, Graph)."""
    rng = np.random.default_rng(seed)
    fam = int(rng.integers(0, len(FAMILIES)))
    n = int(2 ** rng.uniform(lo, hi))
    if fam == 6:
        k = int(rng.integers(2, 9))
        sizes = np.maximum(16, (n * rng.dirichlet(np.ones(k))).astype(int))
        g = inputs.disjoint_union([_member(rng, s) for s in sizes])
    else:
        g = _family_graph(fam, n, rng)
    return FAMILIES[fam], g


def time_arm(ctx, csr, v, labels, ncomp, reps=3, slow_ms=20.0):
    """Median device time (ms) of one arm; None-safe censoring at the round limit."""
    def once():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        censored = False
        try:
            b.connectivity_csr(ctx, csr, v, labels=labels, ncomp=ncomp)
        except b.CCError as e:
            if e.status != b.CC_ELIVELOCK:
                raise
            censored = True
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), censored

    t, cens = once()
    if cens or t > slow_ms:
        return t, cens
    ts = [t] + [once()[0] for _ in range(reps - 1)]
    return statistics.median(ts), False


def measure(ctx, g, arm_list, reps=3):
    dev = ctx.torch_device
    csr = b.build_csr(ctx, g.n, g.u, g.v, dedup=True)
    feats = b.graph_features(ctx, csr)
    labels = torch.empty(csr.n, dtype=torch.int32, device=dev)
    ncomp = torch.empty(1, dtype=torch.int64, device=dev)
    times, cens = [], []
    for v in arm_list:
        t, c = time_arm(ctx, csr, v, labels, ncomp, reps)
        times.append(t)
        cens.append(c)
    return csr, feats, times, cens


def build_corpus(ctx, seeds, lo=12, hi=22, round_limit=2000, log=None, reps=3):
    """Features and per-arm times for the given seeds (graphs generated on the
    host in a background thread while the GPU times the previous one)."""
    ctx.set_round_limit(round_limit)
    arm_list = arms()
    rows = []
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=1) as ex:
        fut = ex.submit(corpus_graph, seeds[0], lo, hi) if seeds else None
        for i, s in enumerate(seeds):
            fam, g = fut.result()
            if i + 1 < len(seeds):
                fut = ex.submit(corpus_graph, seeds[i + 1], lo, hi)
            _, feats, times, cens = measure(ctx, g, arm_list, reps)
            rows.append(dict(seed=s, family=fam, n=g.n, pairs=g.num_pairs, features=feats, times=times,
                             censored=cens))
            if log and (i % 10 == 0 or i + 1 == len(seeds)):
                log(f"corpus {i + 1}/{len(seeds)} seed={s} {fam} n={g.n} best={int(np.argmin(times))} "
                    f"t={min(times):.3f}ms elapsed={time.time() - t0:.0f}s")
    ctx.set_round_limit(0)
    return rows


def targets(times):
    t = np.asarray(times, np.float64)
    return np.log(t) - np.log(t.min(axis=1, keepdims=True))


def normaliser(X):
    X = np.asarray(X, np.float64)
    mu = X.mean(0)
    sd = X.std(0)
    sd[sd < 1e-6] = 1.0
    return np.concatenate([mu, sd]).astype(np.float32)


def init_params(K: int, seed: int = 0):
    """Glorot-uniform weights, zero biases (FP32 master copy)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((16, 64), (64, 64), (64, K)):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def train(ctx, X, Y, epochs=300, batch=64, lr=2e-3, seed=0, log=None):
    """Adam on the GPU with the library's forward / backward / Adam kernels.
    X: normalised features [N,16]; Y: targets [N,K].  Returns (params_bf16
    device tensor, FP32 master numpy, loss history)."""
    dev = ctx.torch_device
    N, K = Y.shape
    master = torch.from_numpy(init_params(K, seed)).to(dev)
    params = b.mlp_pack_bf16(master)
    m1 = torch.zeros_like(master)
    m2 = torch.zeros_like(master)
    Xd = torch.from_numpy(np.asarray(X, np.float32)).to(dev)
    Yd = torch.from_numpy(np.asarray(Y, np.float32)).to(dev)
    cache = torch.empty(batch * 256, dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(N)).to(dev)
        losses = []
        for s0 in range(0, N, batch):
            idx = perm[s0:s0 + batch]
            xb = Xd[idx].contiguous()
            yb = Yd[idx].contiguous()
            out = b.mlp_forward(params, K, xb, cache)
            g, loss = b.mlp_backward(params, K, xb, cache, out, yb)
            step += 1
            b.mlp_adam(master, params, g, m1, m2, lr, 0.9, 0.999, 1e-8, step)
            losses.append(loss)
        ep_loss = float(torch.stack(losses).mean().item())
        hist.append(ep_loss)
        if log and (ep % 50 == 0 or ep + 1 == epochs):
            log(f"epoch {ep} loss {ep_loss:.4f}")
    return params, master.cpu().numpy(), hist


def predict(ctx, params, K, Xn):
    Xd = torch.from_numpy(np.asarray(Xn, np.float32)).to(ctx.torch_device)
    return b.mlp_forward(params, K, Xd).cpu().numpy()


def save(path, master, norm, K, gate=(0, -1), meta=None):
    np.savez(path, master=master, norm=norm, K=np.int32(K), gate_vertices=np.int64(gate[0]),
             gate_arm=np.int32(gate[1]), **(meta or {}))


def load(ctx, path):
    """(params_bf16 on the device, norm, K, gate)."""
    z = np.load(path, allow_pickle=False)
    master = torch.from_numpy(z["master"].astype(np.float32)).to(ctx.torch_device)
    gate = (int(z["gate_vertices"]), int(z["gate_arm"])) if "gate_vertices" in z.files else (0, -1)
    return b.mlp_pack_bf16(master), z["norm"].astype(np.float32), int(z["K"]), gate


def evaluate(ctx, params, norm, seeds, lo=12, hi=22, reps=3, log=None, gate=(0, -1), all80=True):
    """Held-out evaluation: time the selector (gate, features, model and
    chosen arm, end to end), the per-graph best arm re-timed independently,
    the fixed default and the decision-tree rules; with all80 also every one
    of the 80 sampling x finish variants of the main table, and the best of
    them re-timed.  Labels of the selector are checked against the
    default's."""
    arm_list = arms()
    main80 = b.all_variants()
    dev = ctx.torch_device
    rows = []
    sel = b.Selector(ctx, params, arm_list, norm, gate=gate)
    ctx.set_round_limit(2000)
    for i, s in enumerate(seeds):
        fam, g = corpus_graph(s, lo, hi)
        csr, feats, times, cens = measure(ctx, g, arm_list, reps)
        best = int(np.argmin(times))
        labels = torch.empty(csr.n, dtype=torch.int32, device=dev)
        ncomp = torch.empty(1, dtype=torch.int64, device=dev)
        # end-to-end selector time (median of reps): features, model and arm
        ts, chosen = [], -1
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            chosen = sel.connectivity(csr, labels, ncomp)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        t_sel = statistics.median(ts[1:])
        sel_labels = labels.cpu().numpy().copy()
        ref, _ = b.connectivity_csr(ctx, csr, arm_list[default_arm_index()], labels=labels, ncomp=ncomp)
        same = bool(np.array_equal(sel_labels, ref.cpu().numpy()))
        t_best, _ = time_arm(ctx, csr, arm_list[best], labels, ncomp, reps)        # re-timed
        t_def = times[default_arm_index()]
        t_tree = times[decision_tree_arm(feats)]
        row = dict(seed=s, family=fam, n=g.n, chosen=chosen, best=best, t_selector=t_sel, t_best=t_best,
                   t_default=t_def, t_tree=t_tree, t_chosen_arm=times[chosen], labels_equal=same,
                   gated=bool(gate[0] > 0 and g.n < gate[0]))
        if all80:
            t80 = [time_arm(ctx, csr, v, labels, ncomp, reps)[0] for v in main80]
            b80 = int(np.argmin(t80))
            row["best80"] = b80
            row["t_best80"], _ = time_arm(ctx, csr, main80[b80], labels, ncomp, reps)    # re-timed
        rows.append(row)
        if log and (i % 10 == 0 or i + 1 == len(seeds)):
            log(f"eval {i + 1}/{len(seeds)} {fam} n={g.n} chosen={chosen} best={best} sel={t_sel:.3f} "
                f"best={t_best:.3f} default={t_def:.3f}")
    ctx.set_round_limit(0)
    return rows


def summarize(rows):
    sel = np.array([r["t_selector"] for r in rows])
    best = np.array([r["t_best"] for r in rows])
    de = np.array([r["t_default"] for r in rows])
    tree = np.array([r["t_tree"] for r in rows])
    arm = np.array([r["t_chosen_arm"] for r in rows])
    out80 = {}
    if rows and "t_best80" in rows[0]:
        b80 = np.array([r["t_best80"] for r in rows])
        out80 = {"best_of_80_variants_ms": float(b80.mean()), "selector_over_best80": float(sel.mean() / b80.mean())}
    return {
        **out80,
        "gated_graphs": int(sum(1 for r in rows if r.get("gated"))),
        "graphs": len(rows),
        "mean_ms": {"selector": float(sel.mean()), "best": float(best.mean()), "default": float(de.mean()),
                    "decision_tree": float(tree.mean()), "chosen_arm_only": float(arm.mean())},
        "selector_over_best": float(sel.mean() / best.mean()),
        "selector_over_default": float(sel.mean() / de.mean()),
        "tree_over_best": float(tree.mean() / best.mean()),
        "picked_best_fraction": float(np.mean([r["chosen"] == r["best"] for r in rows])),
        "labels_always_equal": bool(all(r["labels_equal"] for r in rows)),
    }


def _log(msg):
    print("[selector]", msg, file=sys.stderr, flush=True)


def _rows_to_npz(rows, path):
    np.savez(path,
             seeds=np.array([r["seed"] for r in rows], np.int64),
             family=np.array([FAMILIES.index(r["family"]) for r in rows], np.int32),
             n=np.array([r["n"] for r in rows], np.int64),
             pairs=np.array([r["pairs"] for r in rows], np.int64),
             features=np.array([r["features"] for r in rows], np.float32),
             times=np.array([r["times"] for r in rows], np.float64),
             censored=np.array([r["censored"] for r in rows], bool))


def load_corpus(paths):
    zs = [np.load(p, allow_pickle=False) for p in paths]
    keys = ("seeds", "family", "n", "pairs", "features", "times", "censored")
    return {k: np.concatenate([z[k] for z in zs]) for k in keys}


def main(argv=None):
    import argparse
    import json
    import os

    ap = argparse.ArgumentParser(prog="python -m paper_2008_03909_amd.selector")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("corpus", help="time every arm on a range of corpus seeds")
    c.add_argument("--seeds", required=True, help="lo:hi (half open)")
    c.add_argument("--out", required=True)
    c.add_argument("--lo", type=int, default=12)
    c.add_argument("--hi", type=int, default=22)
    t = sub.add_parser("train", help="train on the non-held-out rows of corpus files")
    t.add_argument("--corpus", nargs="+", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--epochs", type=int, default=400)
    e = sub.add_parser("eval", help="end-to-end timing of the trained selector on held-out seeds")
    e.add_argument("--model", required=True)
    e.add_argument("--seeds", required=True, help="lo:hi; only seeds with seed %% 10 == 0 are used")
    e.add_argument("--out", required=True)
    e.add_argument("--lo", type=int, default=12)
    e.add_argument("--hi", type=int, default=22)
    e.add_argument("--no-all80", action="store_true", help="skip timing the 80 main variants per graph")
    g2 = sub.add_parser("gate", help="fit the small-graph gate of an existing model from corpus files")
    g2.add_argument("--model", required=True)
    g2.add_argument("--corpus", nargs="+", required=True)
    a = ap.parse_args(argv)
    ctx = b.Context(0)
    if a.cmd == "corpus":
        lo, hi = (int(x) for x in a.seeds.split(":"))
        rows = build_corpus(ctx, list(range(lo, hi)), a.lo, a.hi, log=_log)
        _rows_to_npz(rows, a.out)
    elif a.cmd == "train":
        C = load_corpus(a.corpus)
        train_mask = C["seeds"] % 10 != 0
        X = C["features"][train_mask]
        norm = normaliser(X)
        Xn = (X - norm[:16]) / norm[16:]
        Y = targets(C["times"][train_mask])
        params, master, hist = train(ctx, Xn, Y, epochs=a.epochs, log=_log)
        K = Y.shape[1]
        keep = prune_arms(predict(ctx, params, K, Xn), C["times"][train_mask])
        master = apply_pruning(master, K, keep)
        params = b.mlp_pack_bf16(torch.from_numpy(master).to(ctx.torch_device))
        _log(f"arms kept: {np.flatnonzero(keep).tolist()}")
        picks_tr = predict(ctx, params, K, Xn).argmin(1)
        gate = choose_gate(C["times"][train_mask], C["n"][train_mask], picks_tr)
        _log(f"gate: graphs below {gate[0]} vertices run arm {gate[1]} without the model")
        save(a.out, master, norm, K, gate, {"loss": np.array(hist, np.float32)})
        # selection quality on the held-out corpus rows (recorded times)
        hm = ~train_mask
        if hm.any():
            Xh = (C["features"][hm] - norm[:16]) / norm[16:]
            pick = predict(ctx, params, K, Xh).argmin(1)
            th = C["times"][hm]
            sel = th[np.arange(th.shape[0]), pick].mean()
            _log(f"held-out rows={hm.sum()} selected/best={sel / th.min(1).mean():.3f} "
                 f"selected/default={sel / th[:, default_arm_index()].mean():.3f}")
    elif a.cmd == "gate":
        C = load_corpus(a.corpus)
        tm = C["seeds"] % 10 != 0
        params, norm, K, _ = load(ctx, a.model)
        Xn = (C["features"][tm] - norm[:16]) / norm[16:]
        picks_tr = predict(ctx, params, K, Xn).argmin(1)
        gate = choose_gate(C["times"][tm], C["n"][tm], picks_tr)
        z = dict(np.load(a.model, allow_pickle=False))
        z["gate_vertices"], z["gate_arm"] = np.int64(gate[0]), np.int32(gate[1])
        np.savez(a.model, **z)
        _log(f"gate: graphs below {gate[0]} vertices run arm {gate[1]} without the model")
    else:
        params, norm, K, gate = load(ctx, a.model)
        lo, hi = (int(x) for x in a.seeds.split(":"))
        seeds = [s for s in range(lo, hi) if s % 10 == 0]
        rows = evaluate(ctx, params, norm, seeds, a.lo, a.hi, log=_log, gate=gate, all80=not a.no_all80)
        out = {"summary": summarize(rows), "rows": rows}
        with open(a.out, "w") as f:
            json.dump(out, f, indent=1)
        _log(json.dumps(out["summary"]))
    ctx.close()


if __name__ == "__main__":
    main()
