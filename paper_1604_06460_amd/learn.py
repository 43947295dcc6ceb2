"""Training data from self-measured timings, fitting, and the learned-vs-plain
comparison for batches.

Orchestration only: features, plans, the batched launch, the per-segment
timings (in-kernel real-time counter) and the model's forward, backward and
Adam steps all run inside libqs.
"""
from __future__ import annotations

import numpy as np

from . import qs as Q

PLAIN = {
    "heuristic": Q.QS_POLICY_HEURISTIC,
    "fixed_k2": Q.QS_POLICY_FIXED_K2,
    "fixed_k4": Q.QS_POLICY_FIXED_K4,
    "fixed_k6": Q.QS_POLICY_FIXED_K6,
}


def random_options(kinds, rng):
    """A random valid option per segment (emulation only for subroutines)."""
    hi = np.where(kinds == Q.QS_SEG_GATES, 3, 4)
    return (rng.random(kinds.size) * hi).astype(np.int32)


def _say(log, msg):
    if log is not None:
        log(msg)


def explore_options(base, kinds, rng, frac):
    """`base` with a random fraction `frac` of its segments given a random
    valid option: plans near a sensible one, so that the timed segments run
    among neighbours like those of the plans that will be chosen later."""
    o = np.array(base, dtype=np.int32, copy=True)
    flip = rng.random(o.size) < frac
    o[flip] = random_options(kinds[flip], rng)
    return o


def collect(batch, runs, seed, with_policies=True, frac=0.35, log=None):
    """Run `batch` under the plain policies (if `with_policies`) and `runs`
    perturbations of them, and return (X, T, mask): features, mean
    natural-log device microseconds per option, and which options were
    measured."""
    rng = np.random.default_rng(seed)
    kinds, _, _ = batch.segment_info()
    X = batch.features()
    n = batch.n_segments
    s = np.zeros((n, 4))
    c = np.zeros((n, 4))
    bases = [Q.choose(batch, p) for p in PLAIN.values()]
    plans = list(bases) if with_policies else []
    plans += [explore_options(bases[i % len(bases)], kinds, rng, frac) for i in range(runs)]
    idx = np.arange(n)
    for pi, opts in enumerate(plans):
        batch.set_plan(opts)
        batch.run()                      # first run after a plan: warm
        ms, seg_us, _, _ = batch.run()
        s[idx, opts] += np.log(np.maximum(seg_us, 1e-3))
        c[idx, opts] += 1
        _say(log, "timing run %d/%d: %.1f ms" % (pi + 1, len(plans), ms))
    mask = (c > 0).astype(np.float32)
    T = np.where(c > 0, s / np.maximum(c, 1), 0.0).astype(np.float32)
    return X, T, mask


def fit(X, T, mask, epochs=80, batch=256, lr=2e-3, seed=0):
    """Standardise the features and train the model with Adam. A feature
    that does not vary over the training rows (up to float rounding, e.g.
    the batch-level size on a single training batch) is switched off: the
    model cannot learn its effect, and scaling rounding noise up would turn
    a different value at inference into a huge input."""
    X64 = X.astype(np.float64)
    mean = X64.mean(0)
    std = X64.std(0)
    inv = np.where(std > 1e-4 * np.maximum(1.0, np.abs(mean)), 1.0 / np.maximum(std, 1e-30), 0.0)
    m = Q.Mlp(seed=seed)
    m.set_norm(mean, inv)
    # training range per feature: the learned policy falls back to the
    # heuristic for segments outside it; switched-off features are not checked
    lo = np.where(inv > 0, X64.min(0), -3.0e38)
    hi = np.where(inv > 0, X64.max(0), 3.0e38)
    m.set_range(lo, hi)
    loss = m.train(X, T, mask, epochs, batch, lr, seed)
    return m, loss


def wall_times(batch, model, repeats=3, log=None):
    """Median wall time (ms) of one launch per policy, and the plans."""
    res, plans = {}, {}
    pols = dict(PLAIN)
    if model is not None:
        pols = {"learned": Q.QS_POLICY_LEARNED, **pols}
    for name, pol in pols.items():
        opts = Q.choose(batch, pol, model if pol == Q.QS_POLICY_LEARNED else None)
        batch.set_plan(opts)
        batch.run()
        res[name] = float(np.median([batch.run()[0] for _ in range(repeats)]))
        plans[name] = opts
        _say(log, "policy %s: %.1f ms" % (name, res[name]))
    return res, plans


def learned_vs_plain(res):
    best = min(v for k, v in res.items() if k != "learned")
    best_name = min((v, k) for k, v in res.items() if k != "learned")[1]
    return res["learned"] / best, best_name
