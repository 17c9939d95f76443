"""Writes the stored expected values for the full-size parity tests.

The heavy-tailed (100,000 nodes, 5,000 cycles, 200,000 faults) and large
(200,000 nodes, 10,000 cycles, 1,000,000 faults) workloads are too big for the
oracle to finish inside a test, so the oracle runs once, here, on a seeded
sample of each fault list: 2,000 faults drawn uniformly without replacement
plus the first 200 faults, in list order, whose site is a register (the
faults most likely to stay latent in state).  Each output file records a
digest of the workload it was computed on, then one line per sampled fault:
its index in the fault list, its first detect cycle (4294967295 = never) and
its event count, with dropping on.

Only the oracle and the seeded input generators are used.

    python tests/golden/make_expected.py [heavy_tailed] [large]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2508_16376_amd import workloads as W  # noqa: E402

SAMPLE_UNIFORM = 2000
SAMPLE_REGISTER = 200


def workload_digest(w) -> str:
    h = hashlib.sha1()
    h.update(np.ascontiguousarray(w.design.nodes).tobytes())
    h.update(np.ascontiguousarray(w.design.po).tobytes())
    h.update(np.ascontiguousarray(w.stimulus).tobytes())
    h.update(np.ascontiguousarray(w.faults).tobytes())
    h.update(str(w.T).encode())
    return h.hexdigest()[:20]


def sample_indices(w, seed: int) -> np.ndarray:
    F = w.faults.size
    perm = np.argsort(W.counter_values(seed, 0, F), kind="stable")
    uni = perm[:SAMPLE_UNIFORM]
    is_reg = w.design.nodes["op"][w.faults["site"]] == W.REG
    regs = np.flatnonzero(is_reg)[:SAMPLE_REGISTER]
    return np.unique(np.concatenate([uni, regs]))


MAKERS = {"heavy_tailed": (W.heavy_tailed, 0x5A3B1E01), "large": (W.large, 0x5A3B1E02)}


def path_for(name: str) -> str:
    return os.path.join(HERE, f"{name}_sample.txt")


def write(name: str):
    make, seed = MAKERS[name]
    t0 = time.time()
    w = make()
    idx = sample_indices(w, seed)
    print(f"{name}: workload in {time.time() - t0:.1f}s, {idx.size} sampled faults", flush=True)
    t0 = time.time()
    G = oracle.golden(w.design, w.stimulus, w.T)
    print(f"{name}: oracle golden trace in {time.time() - t0:.1f}s", flush=True)
    t0 = time.time()
    det, ev = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults[idx], G=G, drop=True, variant=1)
    print(f"{name}: oracle O1 on the sample in {time.time() - t0:.1f}s", flush=True)
    with open(path_for(name), "w") as f:
        f.write(f"# workload {name} digest {workload_digest(w)}\n")
        f.write("# index detect events (oracle O1, drop on)\n")
        for i, d, e in zip(idx, det, ev):
            f.write(f"{int(i)} {int(d)} {int(e)}\n")


def read(name: str):
    """(digest, index, detect, events) of a stored sample."""
    with open(path_for(name)) as f:
        digest = f.readline().split()[-1]
        rows = np.loadtxt(f, dtype=np.uint64, comments="#", ndmin=2)
    return digest, rows[:, 0].astype(np.int64), rows[:, 1].astype(np.uint32), rows[:, 2]


if __name__ == "__main__":
    for n in sys.argv[1:] or list(MAKERS):
        write(n)
