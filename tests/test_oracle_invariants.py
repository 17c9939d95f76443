"""Invariants of fault simulation checked on the oracle, and O0 against O1."""
import numpy as np
import pytest

import oracle
from helpers import Builder, faults
from paper_2508_16376_amd import workloads as W

UND = oracle.UNDETECTED


def _seq_fanin_cone(d):
    """Nodes from which some primary output is reachable (through registers too)."""
    N = d.num_nodes
    preds = [[] for _ in range(N)]
    for n in range(N):
        op = int(d.nodes["op"][n])
        if op in (W.CONST, W.PI):
            continue
        for k in range(W.ARITY[op]):
            preds[n].append(int(d.nodes[f"in{k}"][n]))
    seen = np.zeros(N, dtype=bool)
    stack = [int(p) for p in d.po]
    while stack:
        n = stack.pop()
        if seen[n]:
            continue
        seen[n] = True
        stack.extend(preds[n])
    return seen


@pytest.fixture(scope="module")
def small():
    w = W.medium(seed=4242, F=1500, T=300, n_nodes=1500)
    G = oracle.golden(w.design, w.stimulus, w.T)
    return w, G


@pytest.fixture(scope="module")
def tiny_run():
    w = W.tiny()
    G = oracle.golden(w.design, w.stimulus, w.T)
    return w, G


def test_o0_equals_o1_tiny_full(tiny_run):
    w, G = tiny_run
    for drop in (True, False):
        d0, e0 = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G, variant=0, drop=drop)
        d1, e1 = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G, variant=1, drop=drop)
        np.testing.assert_array_equal(d0, d1)
        np.testing.assert_array_equal(e0, e1)


def test_o0_equals_o1_small_layered(small):
    w, G = small
    for drop in (True, False):
        d0, e0 = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults[:400], G=G, variant=0, drop=drop)
        d1, e1 = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults[:400], G=G, variant=1, drop=drop)
        np.testing.assert_array_equal(d0, d1)
        np.testing.assert_array_equal(e0, e1)


def test_detect_range_and_drop_independence(small):
    w, G = small
    d1, e1 = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G, drop=True)
    dn, en = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G, drop=False)
    np.testing.assert_array_equal(d1, dn)
    assert ((d1 < w.T) | (d1 == UND)).all()
    assert (e1 <= en).all()
    assert (e1[d1 == UND] == en[d1 == UND]).all()
    # both populations are present, so the checks above are not vacuous
    assert (d1 == UND).sum() > 0 and (d1 != UND).sum() > 0


def test_first_excitation_lower_bound(small):
    """Nothing diverges before the site's golden bit first differs from the stuck value."""
    w, G = small
    det, ev = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G, drop=False)
    s = w.faults["site"].astype(np.int64)
    b = w.faults["bit"].astype(np.uint64)
    v = w.faults["stuck"].astype(np.uint64)
    bits = (G[:, s] >> b[None, :]) & np.uint64(1)          # [T][F]
    exc = bits != v[None, :]
    first = np.where(exc.any(axis=0), exc.argmax(axis=0), UND)
    det_ok = det != UND
    assert (det[det_ok] >= first[det_ok]).all()
    never = ~exc.any(axis=0)
    assert (det[never] == UND).all() and (ev[never] == 0).all()


def test_outside_fanin_cone_never_detected(tiny_run):
    w, G = tiny_run
    cone = _seq_fanin_cone(w.design)
    outside = [n for n in range(w.design.num_nodes) if not cone[n] and w.design.nodes["op"][n] != W.PI]
    rows = []
    for n in outside[:50]:
        for bit in range(int(w.design.nodes["width"][n])):
            rows += [(n, bit, 0), (n, bit, 1)]
    assert rows, "the tiny design has dangling logic, so this check is not vacuous"
    det, _ = oracle.fault_sim(w.design, w.stimulus, w.T, faults(rows), G=G)
    assert (det == UND).all()


def test_unobservable_by_construction():
    """A node outside every output cone, and a bit tied to the stuck value."""
    b = Builder()
    a = b.pi(8)
    c = b.pi(8)
    r = b.reg(8)
    x = b.node(W.XOR, 8, (a, r))
    b.set_d(r, x)
    dead = b.node(W.ADD, 8, (x, c))                # read by nobody
    zero = b.const(8, 0)
    anded = b.node(W.AND, 8, (c, zero))            # always 0
    out = b.node(W.OR, 8, (x, anded))
    d = b.design([out])
    T = 200
    stim = W.counter_values(9, 0, 2 * T).reshape(T, 2) & np.uint64(255)
    rows = [(dead, k, v) for k in range(8) for v in (0, 1)] + [(anded, k, 0) for k in range(8)]
    for variant in (0, 1):
        det, ev = oracle.fault_sim(d, stim, T, faults(rows), variant=variant)
        assert (det == UND).all()
        # stuck-at-0 on a bit that is 0 in every cycle never diverges
        assert (ev[16:] == 0).all()


def test_po_bit_exactly_one_polarity_at_cycle_zero(small):
    w, G = small
    rows = []
    for p in w.design.po[:16]:
        for bit in range(int(w.design.nodes["width"][p])):
            rows += [(int(p), bit, 0), (int(p), bit, 1)]
    det, _ = oracle.fault_sim(w.design, w.stimulus, w.T, faults(rows), G=G)
    pair = det.reshape(-1, 2)
    assert (((pair[:, 0] == 0) ^ (pair[:, 1] == 0))).all()


def test_t_prefix(small):
    w, G = small
    full, _ = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G)
    Tp = w.T // 3
    part, _ = oracle.fault_sim(w.design, w.stimulus, Tp, w.faults, G=G[:Tp])
    want = np.where(full < Tp, full, UND)
    np.testing.assert_array_equal(part, want)


def test_node_order_does_not_matter(tiny_run):
    w, G = tiny_run
    N = w.design.num_nodes
    perm = np.array(W.counter_values(31, 0, N).argsort(), dtype=np.int64)
    from helpers import permute_design
    dp = permute_design(w.design, perm)
    fl = w.faults.copy()
    fl["site"] = perm[fl["site"].astype(np.int64)]
    d0, e0 = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G)
    d1, e1 = oracle.fault_sim(dp, w.stimulus, w.T, fl)
    np.testing.assert_array_equal(d0, d1)
    np.testing.assert_array_equal(e0, e1)


def test_thread_count_does_not_matter(small):
    w, G = small
    a = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G, nthreads=1)
    b = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, G=G, nthreads=7)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_flips_o0_equals_o1_and_bounds(small, tiny_run):
    """Bit flips: O0 and O1 agree; nothing is detected before the flip cycle;
    a flip at or after the last cycle changes nothing; drop never changes detect."""
    for w, G in (tiny_run, small):
        fl = W.gen_flip_faults(99, w.design, 600, w.T + 40)      # some flips land at or after T
        for drop in (True, False):
            d0, e0 = oracle.fault_sim(w.design, w.stimulus, w.T, fl, G=G, variant=0, drop=drop)
            d1, e1 = oracle.fault_sim(w.design, w.stimulus, w.T, fl, G=G, variant=1, drop=drop)
            np.testing.assert_array_equal(d0, d1)
            np.testing.assert_array_equal(e0, e1)
        t0 = fl["t0"].astype(np.int64)
        late = t0 >= w.T
        assert late.any() and (~late).any()
        assert (d1[late] == UND).all() and (e1[late] == 0).all()
        det = d1 != UND
        assert (d1[det].astype(np.int64) >= t0[det]).all()
        # every flip before T changes its site for one cycle: at least one event
        assert (e1[~late] >= 1).all()
        dd, _ = oracle.fault_sim(w.design, w.stimulus, w.T, fl, G=G, variant=1, drop=True)
        np.testing.assert_array_equal(dd, d1)
