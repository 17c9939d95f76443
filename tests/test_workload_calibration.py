"""The heavy-tailed workload has the shape its description asks for, measured
with the oracle on a seeded sample of its fault list (a property of the
seeded input generator, not of the simulator):

  - about 2% of the faults stay latent: undetected, with some register state
    still divergent in the last cycle;
  - nearly all others (about 98% in all) are detected within the first ten
    cycles, or leave no divergent register state from cycle 10 on.

The late remainder are faults whose only path to an output passes a
multiplexer leg that an input selects half the time.
"""
import numpy as np

import oracle
from paper_2508_16376_amd import workloads as W

UND = oracle.UNDETECTED


def test_heavy_tailed_latent_and_early_shares():
    w = W.heavy_tailed()
    n = 4000
    idx = np.sort(np.argsort(W.counter_values(0xCA11B, 0, w.faults.size), kind="stable")[:n])
    det, _, _, last_reg = oracle.fault_sim_stats(w.design, w.stimulus, w.T, w.faults[idx])
    und = det == UND
    latent = und & (last_reg == w.T - 1)
    early = (det <= 9) | (und & ((last_reg == UND) | (last_reg < 10)))
    print(f"latent {latent.mean():.4f}, early {early.mean():.4f}")
    assert 0.015 <= latent.mean() <= 0.025
    assert early.mean() >= 0.96
    assert latent.mean() + early.mean() >= 0.98
