"""What the trained selector gains over the method without it, on the CPU
from committed data: the network trained on the GPU
(paper_2008_03909_amd/selector_data/model.npz) is applied by the oracle's
MLP forward pass to the recorded features of the 200 held-out corpus graphs
(seed % 10 == 0); the recorded time of each selected arm is compared with
the per-graph best arm, the fixed default (k-out + UF-Rem-CAS /
SplitAtomicOne / FindNaive) and the paper's text rules.  The end-to-end
figures of the GPU evaluation (selector_data/eval.json: the selector's own
time -- gate, features, forward pass, host wait and chosen arm -- against
the best arm and the best of the 80 main variants, each re-timed) are
checked too."""
import json
import glob
import os

import numpy as np

from oracle import mlp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DATA = os.path.join(ROOT, "paper_2008_03909_amd", "selector_data")
DEFAULT_ARM = 4


def _corpus():
    zs = [np.load(p, allow_pickle=False) for p in sorted(glob.glob(os.path.join(DATA, "corpus_*.npz")))]
    assert zs, "no committed corpus"
    return {k: np.concatenate([z[k] for z in zs]) for k in ("seeds", "features", "times")}


def _picks(features):
    z = np.load(os.path.join(DATA, "model.npz"), allow_pickle=False)
    K, norm = int(z["K"]), z["norm"].astype(np.float64)
    sd = np.where(norm[16:] > 0, norm[16:], 1.0)
    x = (features.astype(np.float32) - norm[:16].astype(np.float32)) / sd.astype(np.float32)
    y, _ = mlp.forward(mlp.bf16_round(z["master"]), x.astype(np.float64), K)
    return y.argmin(1)


def test_corpus_shape():
    C = _corpus()
    assert C["seeds"].size == 2000 and np.unique(C["seeds"]).size == 2000
    assert np.sum(C["seeds"] % 10 == 0) == 200
    assert C["times"].shape[0] == 2000 and C["times"].shape[1] >= 16 and np.all(C["times"] > 0)


def test_trained_selector_against_best_default_and_rules():
    """On recorded times each entry is one median of three runs, and a few
    were disturbed (one arm of one held-out graph recorded 29 ms against a
    0.33 ms re-timing), so entries are clipped at 5x their row's median; the
    recorded per-graph minimum is the smallest of 24 such measurements and
    so biased low, which the end-to-end test below avoids by re-timing."""
    C = _corpus()
    held = C["seeds"] % 10 == 0
    t = C["times"][held]
    t = np.minimum(t, 5.0 * np.median(t, axis=1, keepdims=True))
    pick = _picks(C["features"][held])
    sel = t[np.arange(t.shape[0]), pick].mean()
    best = t.min(1).mean()
    default = t[:, DEFAULT_ARM].mean()
    rules = t[np.arange(t.shape[0]), np.where(C["features"][held][:, 14] > 0.5, 0, DEFAULT_ARM)].mean()
    assert sel <= 1.20 * best, (sel, best)
    assert sel < 0.9 * default, (sel, default)
    assert sel < rules, (sel, rules)


def test_end_to_end_evaluation():
    """The selector's measured end-to-end mean is within 10% of the per-graph
    best arm, at least 5% below the fixed default, and never changes a label; its regret
    against the best of the 80 main variants is reported beside it."""
    d = json.load(open(os.path.join(DATA, "eval.json")))
    s = d["summary"]
    assert s["graphs"] == 200 and s["labels_always_equal"]
    assert s["selector_over_best"] <= 1.10, s
    assert s["selector_over_default"] < 0.95, s
    assert "selector_over_best80" in s and s["selector_over_best80"] < s["mean_ms"]["default"] / s["best_of_80_variants_ms"]
    rows = d["rows"]
    sel = np.mean([r["t_selector"] for r in rows])
    assert abs(sel / np.mean([r["t_best"] for r in rows]) - s["selector_over_best"]) < 1e-9


def test_arm_pruning_drops_an_over_rated_arm():
    """prune_arms removes an arm the model picks where it is slow and keeps
    the arms it picks well; apply_pruning only touches the output biases."""
    from paper_2008_03909_amd import selector as S
    rng = np.random.default_rng(0)
    N, K = 400, 5
    T = 1.0 + 0.05 * rng.random((N, K))
    good = rng.integers(0, 3, N)                  # arms 0..2 are each best on a third
    T[np.arange(N), good] = 0.5
    T[:, 3] = 3.0                                 # arm 3 is always slow ...
    pred = np.log(T) + 0.01 * rng.random((N, K))
    pred[: N // 2, 3] = -1.0                      # ... but the model rates it best on half the rows
    keep = S.prune_arms(pred, T)
    assert not keep[3] and keep[0] and keep[1] and keep[2]
    master = np.arange(20 + K, dtype=np.float32)
    m = S.apply_pruning(master, K, keep)
    assert np.array_equal(m[:20], master[:20])
    assert m[20 + 3] == S.PRUNED_BIAS and np.all(m[20:][keep] == master[20:][keep])
