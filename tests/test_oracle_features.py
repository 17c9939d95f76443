"""Pin the predictor-feature reference on designs with closed-form answers."""
import numpy as np

import oracle
from oracle import features as FT
from helpers import Builder, faults
from paper_2508_16376_amd import workloads as W


def test_counter_toggles_and_excitation():
    n, T = 8, 700
    b = Builder()
    b.pi(1)
    cnt = b.reg(n)
    add = b.node(W.ADD, n, (cnt, b.const(n, 1)))
    b.set_d(cnt, add)
    d = b.design([cnt])
    G = oracle.golden(d, np.zeros((T, 1), dtype=np.uint64), T)
    fl = faults([(cnt, k, 0) for k in range(n)] + [(cnt, k, 1) for k in range(n)])
    f = FT.features(d, G, fl)
    t = np.arange(T)
    for k in range(n):
        # bit k of t changes at every multiple of 2^k
        assert f[k, 4] == (T - 1) // (2 ** k) / (T - 1)
        ones = np.count_nonzero((t >> k) & 1)
        assert f[k, 5] == ones / T             # stuck-at-0 is excited where the bit is 1
        assert f[n + k, 5] == (T - ones) / T
        assert f[k, 3] == 3.0                  # log2(8)
        assert f[k, 2] == 0                    # the register is the output
    # cone of the register: the adder only (the register it feeds is the site itself)
    assert f[0, 0] == np.log2(1 + 1)


def test_delay_line_register_depth_and_unobservable():
    L = 6
    b = Builder()
    x = b.pi(4)
    regs = [b.reg(4) for _ in range(L)]
    b.set_d(regs[0], x)
    for j in range(1, L):
        b.set_d(regs[j], regs[j - 1])
    dead = b.node(W.XOR, 4, (regs[2], x))
    d = b.design([regs[-1]])
    depth = FT.register_depth(d)
    for j, r in enumerate(regs, start=1):
        assert depth[r] == L - j
    assert depth[x] == L
    assert depth[dead] == -1


def test_chain_cones_levels_and_cap():
    b = Builder()
    x = b.pi(8)
    y = b.pi(8)
    chain = [b.node(W.ADD, 8, (x, y))]
    for _ in range(1500):
        chain.append(b.node(W.XOR, 8, (chain[-1], y)))
    r = b.reg(8)
    b.set_d(r, chain[-1])
    d = b.design([r])
    cu, ru = FT._users(d)
    assert FT.cone_size(d, chain[-1], cu, ru) == 1           # only the register
    assert FT.cone_size(d, chain[-3], cu, ru) == 3
    assert FT.cone_size(d, chain[0], cu, ru) == FT.CONE_CAP  # 1501 reachable, capped
    lvl = FT.levels(d)
    assert lvl[chain[0]] == 1 and lvl[chain[-1]] == 1501 and lvl[r] == 0


def test_flip_excitation_is_one_cycle():
    from helpers import faults
    b = Builder()
    x = b.pi(4)
    r = b.reg(4)
    b.set_d(r, x)
    d = b.design([r])
    T = 50
    stim = (np.arange(T, dtype=np.uint64) % np.uint64(16))[:, None]
    G = oracle.golden(d, stim, T)
    f = FT.features(d, G, faults([(r, 1, 2, 10), (r, 1, 2, T), (r, 1, 0, 0)]))
    assert f[0, 5] == 1.0 / T and f[1, 5] == 0.0
    assert f[0, 4] == f[2, 4]          # the toggle rate does not depend on the fault model
