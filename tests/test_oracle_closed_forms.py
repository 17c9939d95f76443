"""Pin the oracle's fault simulation on designs whose detect cycles have closed forms."""
import itertools

import numpy as np
import pytest

import oracle
from bitblast import simulate
from helpers import Builder, all_faults, faults
from paper_2508_16376_amd.workloads import ADD, AND, CONST, OR, REG, XOR, MUX, counter_values

UND = oracle.UNDETECTED


def counter(n, po_is_adder=False):
    """n-bit counter: cnt' = cnt + 1 from reset 0; golden cnt(t) = t mod 2^n."""
    b = Builder()
    x = b.pi(1)                      # unused input, keeps the stimulus non-empty
    cnt = b.reg(n)
    one = b.const(n, 1)
    add = b.node(ADD, n, (cnt, one))
    b.set_d(cnt, add)
    d = b.design([add if po_is_adder else cnt])
    return d, cnt, add, x


@pytest.mark.parametrize("n", [3, 6, 10])
def test_counter_golden_trace(n):
    d, cnt, add, _ = counter(n)
    T = 3000
    G = oracle.golden(d, np.zeros((T, 1), dtype=np.uint64), T)
    t = np.arange(T, dtype=np.uint64)
    np.testing.assert_array_equal(G[:, cnt], t % np.uint64(1 << n))
    np.testing.assert_array_equal(G[:, add], (t + np.uint64(1)) % np.uint64(1 << n))


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("drop", [True, False])
def test_counter_register_faults(variant, drop):
    n, T = 10, 600
    d, cnt, add, _ = counter(n)
    stim = np.zeros((T, 1), dtype=np.uint64)
    fl = faults([(cnt, k, 0) for k in range(n)] + [(cnt, k, 1) for k in range(n)])
    det, ev = oracle.fault_sim(d, stim, T, fl, drop=drop, variant=variant)
    for k in range(n):
        # SA0 on bit k: the state first has bit k set at t = 2^k
        assert det[k] == (2 ** k if 2 ** k < T else UND), k
        # SA1 on bit k: the reset state 0 already differs
        assert det[n + k] == 0


@pytest.mark.parametrize("variant", [0, 1])
def test_counter_adder_faults(variant):
    n, T = 9, 700
    stim = np.zeros((T, 1), dtype=np.uint64)
    for po_is_adder in (False, True):
        d, cnt, add, _ = counter(n, po_is_adder)
        fl = faults([(add, k, 0) for k in range(n)] + [(add, k, 1) for k in range(n)])
        det, _ = oracle.fault_sim(d, stim, T, fl, variant=variant)
        for k in range(n):
            # SA0: the adder output t+1 first has bit k set at t = 2^k - 1
            first = 2 ** k - 1 + (0 if po_is_adder else 1)
            assert det[k] == (first if first < T else UND), (po_is_adder, k)
            # SA1: excited at t = 0 for k >= 1 (1 has bit k clear), at t = 1 for k = 0
            first1 = (0 if k >= 1 else 1) + (0 if po_is_adder else 1)
            assert det[n + k] == first1, (po_is_adder, k)


def delay_line(L, w):
    b = Builder()
    x = b.pi(w)
    regs = [b.reg(w) for _ in range(L)]
    b.set_d(regs[0], x)
    for j in range(1, L):
        b.set_d(regs[j], regs[j - 1])
    return b.design([regs[-1]]), x, regs


@pytest.mark.parametrize("variant", [0, 1])
def test_delay_line(variant):
    L, w, T = 5, 4, 200
    d, x, regs = delay_line(L, w)
    stim = (counter_values(77, 0, T) & np.uint64(15))[:, None]
    po_golden = np.zeros(T, dtype=np.uint64)
    po_golden[L:] = stim[:T - L, 0]
    rows = [(regs[j], b, v) for j in range(L) for b in range(w) for v in (0, 1)]
    det, _ = oracle.fault_sim(d, stim, T, faults(rows), variant=variant)
    G = oracle.golden(d, stim, T)
    np.testing.assert_array_equal(G[:, regs[-1]], po_golden)
    for i, (site, b, v) in enumerate(rows):
        j = regs.index(site) + 1                   # stage number 1..L
        bits = (po_golden >> np.uint64(b)) & np.uint64(1)
        cand = [t for t in range(L - j, T) if int(bits[t]) != v]
        assert det[i] == (cand[0] if cand else UND), (j, b, v)


@pytest.mark.parametrize("variant", [0, 1])
def test_po_node_fault_is_first_excitation(variant):
    """A fault on a primary output's own node is detected at its first excitation,
    also when the output feeds back through registers."""
    b = Builder()
    a = b.pi(8)
    r = b.reg(8)
    s = b.node(XOR, 8, (a, r))
    b.set_d(r, s)
    d = b.design([s])
    T = 300
    stim = (counter_values(5, 0, T) & np.uint64(255))[:, None]
    fl = all_faults(d, [s])
    det, _ = oracle.fault_sim(d, stim, T, fl, variant=variant)
    G = oracle.golden(d, stim, T)
    for i in range(fl.size):
        bit = (G[:, s] >> np.uint64(fl["bit"][i])) & np.uint64(1)
        exc = np.nonzero(bit != fl["stuck"][i])[0]
        assert det[i] == (exc[0] if exc.size else UND)


def test_combinational_exhaustive_first_distinguishing_vector():
    """Purely combinational design, stimulus t = t-th input vector: the detect
    cycle is the index of the first vector on which faulty and good outputs differ
    (computed with the gate-level evaluator)."""
    b = Builder()
    p = [b.pi(2) for _ in range(3)]
    n1 = b.node(ADD, 2, (p[0], p[1]))
    n2 = b.node(AND, 2, (n1, p[2]))
    n3 = b.node(XOR, 2, (n1, p[1]))
    n4 = b.node(MUX, 2, (b.node(XOR, 1, (n2, n3)), n2, n3))
    n5 = b.node(OR, 1, (n4, p[0]))
    d = b.design([n4, n5])
    vecs = np.array(list(itertools.product(range(4), repeat=3)), dtype=np.uint64)
    T = vecs.shape[0]
    fl = all_faults(d, [n for n in range(d.num_nodes)])
    for variant in (0, 1):
        det, _ = oracle.fault_sim(d, vecs, T, fl, variant=variant)
        for i in range(fl.size):
            f = (int(fl["site"][i]), int(fl["bit"][i]), int(fl["stuck"][i]))
            good = simulate(d, vecs[:, None, :])[:, 0, :]
            bad = simulate(d, vecs[:, None, :], f)[:, 0, :]
            diff = (good[:, d.po] != bad[:, d.po]).any(axis=1)
            want = int(np.argmax(diff)) if diff.any() else UND
            assert det[i] == want, (variant, f)


# ---------------------------------------------------------------------------
# Bit flips (a single-event upset of a register, a transient on a wire)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("drop", [True, False])
def test_counter_register_flip(variant, drop):
    """Flipping bit k of the counter state in cycle t0: the output differs at
    t0 and from then on (the state keeps a difference of 2^k modulo 2^n); with
    dropping the events are the register and the adder it feeds, at t0."""
    n, T = 8, 300
    d, cnt, add, _ = counter(n)
    stim = np.zeros((T, 1), dtype=np.uint64)
    rows = [(cnt, k, 2, t0) for k in range(n) for t0 in (0, 1, 37, T - 1, T, 5000)]
    det, ev = oracle.fault_sim(d, stim, T, faults(rows), drop=drop, variant=variant)
    for i, (_, k, _, t0) in enumerate(rows):
        if t0 >= T:
            assert det[i] == UND and ev[i] == 0
            continue
        assert det[i] == t0
        assert ev[i] == (2 if drop else 2 * (T - t0)), (k, t0)


@pytest.mark.parametrize("variant", [0, 1])
def test_counter_adder_flip(variant):
    """A flip of the adder output in cycle t0 reaches the state, so the
    register output differs from t0 + 1 on; the adder output itself at t0."""
    n, T = 8, 300
    stim = np.zeros((T, 1), dtype=np.uint64)
    for po_is_adder in (False, True):
        d, cnt, add, _ = counter(n, po_is_adder)
        rows = [(add, k, 2, t0) for k in range(n) for t0 in (0, 5, 100, T - 1)]
        det, _ = oracle.fault_sim(d, stim, T, faults(rows), variant=variant)
        for i, (_, k, _, t0) in enumerate(rows):
            want = t0 if po_is_adder else (t0 + 1 if t0 + 1 < T else UND)
            assert det[i] == want, (po_is_adder, k, t0)


@pytest.mark.parametrize("variant", [0, 1])
def test_delay_line_flip(variant):
    """A flip at stage j in cycle t0 arrives at the output L - j cycles later,
    whatever the data: d = t0 + L - j when that is before T."""
    L, w, T = 5, 4, 60
    d, x, regs = delay_line(L, w)
    stim = (counter_values(78, 0, T) & np.uint64(15))[:, None]
    rows = [(regs[j], b, 2, t0) for j in range(L) for b in range(w) for t0 in (0, 3, 40, T - 2)]
    rows += [(x, b, 2, t0) for b in range(w) for t0 in (0, 50, T - L)]
    det, ev = oracle.fault_sim(d, stim, T, faults(rows), drop=False, variant=variant)
    for i, (site, b, _, t0) in enumerate(rows):
        j = regs.index(site) + 1 if site in regs else 0     # the input is stage 0
        want = t0 + L - j
        assert det[i] == (want if want < T else UND), (j, b, t0)
        # one divergent node per cycle from t0 through the last stage reached
        assert ev[i] == min(L - j, T - 1 - t0) + 1, (j, b, t0)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("n", [8, 32, 33, 64])
def test_counter_words_closed_form(variant, n):
    """SA1 on a counter register bit, output = the register: detected in cycle
    0, where the register (excited site, no operands) and the adder (two
    operands) are the only events: 2w + 4w words, plus w for the site's golden
    word; w = 2 words for values wider than 32 bits.  No register state has
    diverged by then."""
    T = 50
    d, cnt, add, _ = counter(n)
    stim = np.zeros((T, 1), dtype=np.uint64)
    fl = faults([(cnt, k, 1) for k in (0, n // 2, n - 1)])
    det, ev, words, lastreg = oracle.fault_sim_stats(d, stim, T, fl, variant=variant)
    w = 2 if n > 32 else 1
    np.testing.assert_array_equal(det, 0)
    np.testing.assert_array_equal(ev, 2)
    np.testing.assert_array_equal(words, 7 * w)
    np.testing.assert_array_equal(lastreg, UND)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("w_bits", [8, 32, 40, 64])
def test_delay_line_words_closed_form(variant, w_bits):
    """SA1 on bit 0 of the input of an L-stage delay line fed with zeros: the
    input is excited every cycle, stage j holds the divergence from cycle j on,
    the output (stage L) shows it in cycle L.  Per cycle t <= L: the site's
    word w, the input event 2w, and min(t, L) divergent registers at 4w each
    (event 2w, state read and write 2w); the last divergent register cycle is
    L."""
    L, T = 5, 40
    d, x, regs = delay_line(L, w_bits)
    stim = np.zeros((T, 1), dtype=np.uint64)
    fl = faults([(x, 0, 1)])
    w = 2 if w_bits > 32 else 1
    for drop in (True, False):
        det, ev, words, lastreg = oracle.fault_sim_stats(d, stim, T, fl, drop=drop, variant=variant)
        last = L if drop else T - 1
        ts = np.arange(last + 1)
        assert det[0] == L
        assert ev[0] == int((1 + np.minimum(ts, L)).sum())
        assert words[0] == int((3 * w + 4 * w * np.minimum(ts, L)).sum())
        assert lastreg[0] == last
