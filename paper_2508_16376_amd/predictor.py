"""Load predictor pipeline: training data from the simulator's own runs,
training, prediction, and the prediction-error report.

Targets are log2(1 + events) of each fault, where events are the bad-gate
evaluations the simulator counts (identical in every mode).  Features and the
network run in the HIP library (riros_features, riros_mlp_*); this module only
collects arrays and computes summary statistics.
"""
from __future__ import annotations

import numpy as np

from . import riros
from . import workloads as W

PREDICTOR_SEED = 0x5EED


def samples_from_runs(runs):
    """Features and targets from (design, golden, faults) triples, simulated
    with the plain kernel with fault dropping on (as production runs are)."""
    xs, ys = [], []
    for d, g, fl in runs:
        _, ev, _ = riros.fault_sim(d, g, fl, mode=riros.MODE_PLAIN)
        xs.append(riros.features(d, g, fl))
        ys.append(np.log2(1.0 + ev.astype(np.float64)).astype(np.float32))
    return np.concatenate(xs), np.concatenate(ys)


def shuffle(x, y, seed=PREDICTOR_SEED):
    perm = np.argsort(W.counter_values(seed, 0, x.shape[0]))
    return x[perm], y[perm]


def train(x, y, *, epochs=8, batch=4096, lr=2e-3, seed=PREDICTOR_SEED):
    x, y = shuffle(x, y, seed)
    return riros.mlp_train(x, y, W.mlp_init_weights(seed), epochs=epochs, batch=batch, lr=lr)


def rank(a: np.ndarray) -> np.ndarray:
    """Average ranks (ties share the mean rank)."""
    order = np.argsort(a, kind="mergesort")
    r = np.empty(a.size, dtype=np.float64)
    r[order] = np.arange(a.size, dtype=np.float64)
    sa = a[order]
    i = 0
    while i < a.size:
        j = i
        while j + 1 < a.size and sa[j + 1] == sa[i]:
            j += 1
        if j > i:
            r[order[i:j + 1]] = 0.5 * (i + j)
        i = j + 1
    return r


def load_error(pred: np.ndarray, target: np.ndarray) -> dict:
    """Spearman rank correlation and mean absolute error in log2 units."""
    rp, rt = rank(np.asarray(pred, dtype=np.float64)), rank(np.asarray(target, dtype=np.float64))
    rp -= rp.mean()
    rt -= rt.mean()
    den = np.sqrt((rp * rp).sum() * (rt * rt).sum())
    rho = float((rp * rt).sum() / den) if den > 0 else 0.0
    return {"spearman": rho, "mean_abs_log2": float(np.mean(np.abs(np.asarray(pred, np.float64) - target)))}
