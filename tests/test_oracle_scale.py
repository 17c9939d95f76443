"""O0 against O1 at the full sizes of the benchmark workloads.

O0 evaluates every node of the design in every cycle (the plain
definition); O1 visits only nodes with a divergent input.  Every GPU parity
test at full size compares with O1, so O1 is pinned against O0 here on
stratified samples of each full-size fault list: uniform faults plus the
faults with the most events (the latent ones, which run every cycle and
exercise register state the longest).  Detect cycles, event counts,
byte-model words and the last divergent-register cycle must be identical.
O0 costs N x T node evaluations per undetected fault (2 x 10^9 on the large
design), so the samples are sized to keep this file within a few minutes.
"""
import numpy as np
import pytest

import oracle
from paper_2508_16376_amd import workloads as W


def _stratified(w, G, n_uniform, n_long, pool, seed):
    perm = np.argsort(W.counter_values(seed, 0, w.faults.size), kind="stable")
    uni = perm[:n_uniform]
    cand = perm[n_uniform:n_uniform + pool]
    _, ev = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults[cand], G=G)
    longest = cand[np.argsort(-ev.astype(np.int64), kind="stable")[:n_long]]
    return np.sort(np.concatenate([uni, longest]))


def _o0_equals_o1(w, G, idx):
    fl = w.faults[idx]
    r0 = oracle.fault_sim_stats(w.design, w.stimulus, w.T, fl, G=G, variant=0)
    r1 = oracle.fault_sim_stats(w.design, w.stimulus, w.T, fl, G=G, variant=1)
    for a, b, what in zip(r0, r1, ("detect", "events", "words", "lastreg")):
        np.testing.assert_array_equal(a, b, err_msg=f"{w.name}: {what}")
    return r1


def test_medium_o0_equals_o1():
    """1,000 medium faults: 900 uniform and the 100 with the most events of
    the whole list."""
    w = W.medium()
    G = oracle.golden(w.design, w.stimulus, w.T)
    _, ev = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G)
    perm = np.argsort(W.counter_values(0x0D01, 0, w.faults.size), kind="stable")
    longest = np.argsort(-ev.astype(np.int64), kind="stable")[:100]
    idx = np.unique(np.concatenate([perm[:900], longest]))
    det, _, _, _ = _o0_equals_o1(w, G, idx)
    assert (det == oracle.UNDETECTED).any() and (det != oracle.UNDETECTED).any()


@pytest.mark.parametrize("name,n_uniform,n_long,pool", [("heavy_tailed", 150, 8, 3000), ("large", 60, 4, 2000)])
def test_template_designs_o0_equals_o1(name, n_uniform, n_long, pool):
    w = {"heavy_tailed": W.heavy_tailed, "large": W.large}[name]()
    G = oracle.golden(w.design, w.stimulus, w.T)
    idx = _stratified(w, G, n_uniform, n_long, pool, 0x0D02)
    det, ev, _, lastreg = _o0_equals_o1(w, G, idx)
    # the longest ones are latent: undetected, with state divergent to the end
    assert ((det == oracle.UNDETECTED) & (lastreg == w.T - 1)).sum() >= n_long // 2


def test_campaign_o0_equals_o1():
    """Eight of the 64 campaign designs, from the smallest to the largest:
    20 uniform faults and the 4 with the most events of 400 more, each."""
    picks = [0, 9, 18, 27, 36, 45, 54, 63]
    ws = W.campaign(only=set(picks))
    assert len(ws) == len(picks)
    for w in ws:
        G = oracle.golden(w.design, w.stimulus, w.T)
        idx = _stratified(w, G, 20, 4, 400, 0x0D03)
        _o0_equals_o1(w, G, idx)
