"""Brute force on tiny sequential designs: every stimulus sequence, every fault.

Detect cycles and event counts of the oracle (O0 and O1) are compared with a
count taken directly from two gate-level simulations (good and faulty machine)
of every node in every cycle:
  - a combinational node counts when an operand or its own value differs;
  - a register counts when its D value of the previous cycle differs or its own
    (forced) value differs;
  - with dropping, counting stops after the detect cycle.
The byte-model words and the last cycle with a divergent register state are
taken from the same two traces: per simulated cycle one word for the site, per
event (k + 2) words for a node with k operands (0 for registers, inputs and
constants), and 2 more per register whose D value differed in the previous
cycle (every node here is at most 32 bits wide, one word a value).
"""
import itertools

import numpy as np
import pytest

import oracle
from bitblast import simulate
from helpers import all_faults, all_flip_faults, fault_tuple
from paper_2508_16376_amd.workloads import ARITY, CONST, PI, REG, gen_layered

UND = oracle.UNDETECTED


def tiny_designs():
    out = []
    for s in range(4):
        d = gen_layered(1000 + s, n_nodes=2 + 2 + 9, n_regs=2, n_pi=2, n_po=2, n_levels=4,
                        widths=[1, 2, 3], wweights=[1, 1, 1], name=f"brute{s}")
        # PI widths small enough for exhaustive sequences: 1 and 2 bits
        pis = np.nonzero(d.nodes["op"] == PI)[0]
        d.nodes["width"][pis[0]] = 1
        d.nodes["width"][pis[1]] = 2
        out.append(d)
    # hand-built: XOR, MUL, CONCAT, NOT, NE, EQ, SUB with register feedback
    from helpers import Builder
    from paper_2508_16376_amd.workloads import XOR, MUL, CONCAT, NOT, NE, EQ, SUB
    b = Builder()
    a, c = b.pi(1), b.pi(2)
    r0, r1 = b.reg(2), b.reg(3, init=5)
    x = b.node(XOR, 2, (c, r0))
    m = b.node(MUL, 3, (x, r1))
    cc = b.node(CONCAT, 3, (a, x))
    nt = b.node(NOT, 3, (cc,))
    ne = b.node(NE, 1, (m, nt))
    sb = b.node(SUB, 2, (x, a))
    eq = b.node(EQ, 1, (sb, r0))
    b.set_d(r0, sb)
    b.set_d(r1, m)
    out.append(b.design([ne, eq], "brute-hand"))
    return out


def reference_counts(d, seqs, fault, drop, stats=False):
    """Detect cycle and events per sequence from gate-level traces (stats: also
    the byte-model words and the last cycle with a divergent register)."""
    good = simulate(d, seqs)
    bad = simulate(d, seqs, fault)
    S, T, N = good.shape
    diff = good != bad                          # [S][T][N]
    po = np.asarray(d.po, dtype=np.int64)
    det_any = diff[:, :, po].any(axis=2)
    detect = np.where(det_any.any(axis=1), det_any.argmax(axis=1), UND).astype(np.int64)
    ev_per_t = np.zeros((S, T), dtype=np.int64)
    words_per_t = np.zeros((S, T), dtype=np.int64)
    regdiv = np.zeros((S, T), dtype=bool)
    for n in range(N):
        op = int(d.nodes["op"][n])
        div = diff[:, :, n].copy()
        k = 0
        if op == REG:
            dnode = int(d.nodes["in0"][n])
            state_div = np.zeros((S, T), dtype=bool)
            state_div[:, 1:] = diff[:, :-1, dnode]
            div |= state_div
            regdiv |= state_div
            words_per_t += 2 * state_div
        elif op not in (CONST, PI):
            k = ARITY[op]
            for j in range(k):
                div |= diff[:, :, int(d.nodes[f"in{j}"][n])]
        ev_per_t += div
        words_per_t += (k + 2) * div
    tt = np.arange(T)[None, :]
    live = tt <= detect[:, None] if drop else np.ones((S, T), dtype=bool)
    ev_per_t = np.where(live, ev_per_t, 0)
    if not stats:
        return detect, ev_per_t.sum(axis=1)
    words = np.where(live, words_per_t + 1, 0).sum(axis=1)      # + the site's word each simulated cycle
    rl = np.where(live & regdiv, tt, -1).max(axis=1)
    lastreg = np.where(rl < 0, UND, rl).astype(np.int64)
    return detect, ev_per_t.sum(axis=1), words, lastreg


@pytest.mark.parametrize("didx", range(5))
def test_brute_force_all_sequences(didx):
    d = tiny_designs()[didx]
    T = 4
    bits_per_cycle = 3                           # PI widths 1 and 2
    seqs_int = np.arange(1 << (bits_per_cycle * T), dtype=np.uint64)
    seqs = np.zeros((seqs_int.size, T, 2), dtype=np.uint64)
    for t in range(T):
        chunk = (seqs_int >> np.uint64(bits_per_cycle * t)) & np.uint64(7)
        seqs[:, t, 0] = chunk & np.uint64(1)
        seqs[:, t, 1] = chunk >> np.uint64(1)
    # every stuck-at fault and every bit flip in every cycle
    fl = np.concatenate([all_faults(d), all_flip_faults(d, T)])
    # sample sequences for the oracle loop, but compare every sequence for a few faults
    rng_idx = np.linspace(0, seqs.shape[0] - 1, 256).astype(np.int64)
    for drop in (True, False):
        ref = [reference_counts(d, seqs[rng_idx], fault_tuple(f), drop) for f in fl]
        for j, s in enumerate(rng_idx):
            for variant in (0, 1):
                det, ev = oracle.fault_sim(d, seqs[s], T, fl, drop=drop, variant=variant)
                for i in range(fl.size):
                    assert det[i] == ref[i][0][j], (variant, drop, s, i)
                    assert ev[i] == ref[i][1][j], (variant, drop, s, i)


def test_brute_force_every_sequence_detect_only():
    """All 4096 sequences of 4 cycles for every fault of one design (O1)."""
    d = tiny_designs()[0]
    T = 4
    seqs_int = np.arange(1 << 12, dtype=np.uint64)
    seqs = np.zeros((seqs_int.size, T, 2), dtype=np.uint64)
    for t in range(T):
        chunk = (seqs_int >> np.uint64(3 * t)) & np.uint64(7)
        seqs[:, t, 0] = chunk & np.uint64(1)
        seqs[:, t, 1] = chunk >> np.uint64(1)
    fl = np.concatenate([all_faults(d), all_flip_faults(d, T)])
    ref = np.stack([reference_counts(d, seqs, fault_tuple(f), True)[0] for f in fl], axis=1)   # [S][F]
    got = np.stack([oracle.fault_sim(d, seqs[s], T, fl, variant=1)[0] for s in range(seqs.shape[0])])
    np.testing.assert_array_equal(got.astype(np.int64), ref)


@pytest.mark.parametrize("didx", [0, 4])
def test_brute_force_words_and_last_register(didx):
    """Byte-model words and the last divergent-register cycle of O0 and O1
    against the gate-level traces, drop on and off."""
    d = tiny_designs()[didx]
    T = 4
    seqs_int = np.arange(1 << 12, dtype=np.uint64)
    seqs = np.zeros((seqs_int.size, T, 2), dtype=np.uint64)
    for t in range(T):
        chunk = (seqs_int >> np.uint64(3 * t)) & np.uint64(7)
        seqs[:, t, 0] = chunk & np.uint64(1)
        seqs[:, t, 1] = chunk >> np.uint64(1)
    fl = np.concatenate([all_faults(d), all_flip_faults(d, T)])
    rng_idx = np.linspace(0, seqs.shape[0] - 1, 64).astype(np.int64)
    for drop in (True, False):
        ref = [reference_counts(d, seqs[rng_idx], fault_tuple(f), drop, stats=True) for f in fl]
        for j, s in enumerate(rng_idx):
            for variant in (0, 1):
                det, ev, words, lastreg = oracle.fault_sim_stats(d, seqs[s], T, fl, drop=drop, variant=variant)
                for i in range(fl.size):
                    assert det[i] == ref[i][0][j], (variant, drop, s, i)
                    assert ev[i] == ref[i][1][j], (variant, drop, s, i)
                    assert words[i] == ref[i][2][j], (variant, drop, s, i, "words")
                    assert lastreg[i] == ref[i][3][j], (variant, drop, s, i, "lastreg")
