"""Gate-level (bit-blasted) evaluator used to pin the oracle's word-level semantics.

Every operator is built from single-bit AND/OR/XOR/NOT gates over numpy bool
arrays (one array element per independent stimulus sequence): a ripple-carry
adder, subtraction as a + ~b + 1, a shift-and-add multiplier, comparators from
the subtractor's borrow, shifts and slices as rewiring.  No word-level integer
arithmetic is used for operator semantics, so a mistake in the oracle's
evaluator (a wrong carry, a swapped MUX leg, a shift in the wrong direction)
shows up as a mismatch.
"""
from __future__ import annotations

import numpy as np

from paper_2508_16376_amd.workloads import (ADD, AND, CONCAT, CONST, EQ, MUL, MUX, NE, NOT, OR, PI,
                                            REG, SHL, SHR, SLICE, SUB, ULT, XOR, ARITY)

Bits = list  # list of np.ndarray[bool], least significant bit first


def _zero(S):
    return np.zeros(S, dtype=bool)


def ext(a: Bits, w: int, S: int) -> Bits:
    """Zero-extend or truncate to w bits."""
    return [a[i] if i < len(a) else _zero(S) for i in range(w)]


def full_add(x, y, c):
    s = x ^ y ^ c
    co = (x & y) | (x & c) | (y & c)
    return s, co


def add_bits(a: Bits, b: Bits, cin, w: int):
    out = []
    c = cin
    for i in range(w):
        s, c = full_add(a[i], b[i], c)
        out.append(s)
    return out, c


def op_bits(op: int, w: int, ins: list, widths: list, param: int, S: int) -> Bits:
    """Output bits (w of them) of one operator."""
    if op in (ADD, SUB, AND, OR, XOR, MUL):
        a = ext(ins[0], w, S)
        b = ext(ins[1], w, S)
        if op == ADD:
            return add_bits(a, b, _zero(S), w)[0]
        if op == SUB:
            return add_bits(a, [~x for x in b], np.ones(S, dtype=bool), w)[0]
        if op == AND:
            return [x & y for x, y in zip(a, b)]
        if op == OR:
            return [x | y for x, y in zip(a, b)]
        if op == XOR:
            return [x ^ y for x, y in zip(a, b)]
        # MUL: sum over i of (a AND b_i) << i, truncated to w bits
        acc = [_zero(S) for _ in range(w)]
        for i in range(w):
            partial = [_zero(S)] * i + [x & b[i] for x in a[:w - i]]
            acc = add_bits(acc, partial, _zero(S), w)[0]
        return acc
    if op == NOT:
        return [~x for x in ext(ins[0], w, S)]
    if op == MUX:
        sel = _zero(S)
        for x in ins[0]:
            sel = sel | x
        a = ext(ins[1], w, S)
        b = ext(ins[2], w, S)
        return [(sel & y) | (~sel & x) for x, y in zip(a, b)]
    if op == SHL:
        a = ins[0]
        return [a[i - param] if 0 <= i - param < len(a) else _zero(S) for i in range(w)]
    if op in (SHR, SLICE):
        a = ins[0]
        return [a[i + param] if i + param < len(a) else _zero(S) for i in range(w)]
    if op in (EQ, NE, ULT):
        m = max(widths[0], widths[1])
        a = ext(ins[0], m, S)
        b = ext(ins[1], m, S)
        if op in (EQ, NE):
            same = np.ones(S, dtype=bool)
            for x, y in zip(a, b):
                same = same & ~(x ^ y)
            r = same if op == EQ else ~same
        else:
            # a - b = a + ~b + 1; a < b exactly when there is no carry out
            _, c = add_bits(a, [~x for x in b], np.ones(S, dtype=bool), m)
            r = ~c
        return ext([r], w, S)
    if op == CONCAT:
        a, b = ins[0], ins[1]
        return ext(list(b) + list(a), w, S)
    raise ValueError(op)


def const_bits(value: int, w: int, S: int) -> Bits:
    return [np.full(S, bool((value >> i) & 1)) for i in range(w)]


def word_to_bits(x: np.ndarray, w: int) -> Bits:
    x = np.asarray(x, dtype=np.uint64)
    return [((x >> np.uint64(i)) & np.uint64(1)).astype(bool) for i in range(w)]


def bits_to_word(bits: Bits) -> np.ndarray:
    out = np.zeros(bits[0].shape, dtype=np.uint64)
    for i, b in enumerate(bits):
        out |= b.astype(np.uint64) << np.uint64(i)
    return out


def topo_order(nodes) -> list[int]:
    """Order with every combinational operand before its user (DFS)."""
    N = nodes.size
    state = [0] * N
    order = []
    for root in range(N):
        if state[root]:
            continue
        stack = [(root, 0)]
        while stack:
            n, k = stack.pop()
            op = int(nodes["op"][n])
            comb = op not in (CONST, PI, REG)
            ar = ARITY[op] if comb else 0
            if k == 0:
                if state[n] == 2:
                    continue
                state[n] = 1
            if k < ar:
                stack.append((n, k + 1))
                child = int(nodes[("in0", "in1", "in2")[k]][n])
                if state[child] == 0:
                    stack.append((child, 0))
                continue
            state[n] = 2
            order.append(n)
    return order


def simulate(design, stim_seqs: np.ndarray, fault=None):
    """Gate-level simulation of S independent stimulus sequences.

    stim_seqs: uint64[S][T][num_pi].  fault: None, (site, bit, stuck) for a
    stuck-at gate, or (site, bit, 2, t0) for a bit inverted in cycle t0 only.
    Returns node values uint64[S][T][N] (bit-assembled for comparison only).
    """
    nodes = design.nodes
    S, T, _ = stim_seqs.shape
    N = nodes.size
    order = topo_order(nodes)
    width = [int(x) for x in nodes["width"]]
    state = {}
    for n in range(N):
        if nodes["op"][n] == REG:
            state[n] = const_bits(int(nodes["param"][n]), width[n], S)
    out = np.zeros((S, T, N), dtype=np.uint64)
    for t in range(T):
        val: dict[int, Bits] = {}
        for n in order:
            op = int(nodes["op"][n])
            w = width[n]
            if op == CONST:
                bits = const_bits(int(nodes["param"][n]), w, S)
            elif op == PI:
                bits = word_to_bits(stim_seqs[:, t, int(nodes["param"][n])], w)
            elif op == REG:
                bits = list(state[n])
            else:
                ids = [int(nodes[f"in{k}"][n]) for k in range(ARITY[op])]
                bits = op_bits(op, w, [val[i] for i in ids], [width[i] for i in ids],
                               int(nodes["param"][n]), S)
            if fault is not None and n == fault[0]:
                bits = list(bits)
                if fault[2] == 2:
                    if t == fault[3]:
                        bits[fault[1]] = ~bits[fault[1]]
                else:
                    bits[fault[1]] = np.full(S, bool(fault[2]))
            val[n] = bits
        for n in range(N):
            out[:, t, n] = bits_to_word(val[n])
        for n in state:
            d = int(nodes["in0"][n])
            state[n] = ext(val[d], width[n], S)
    return out


def detect_cycles(design, stim_seqs: np.ndarray, fault) -> np.ndarray:
    """First cycle where a primary output differs (0xFFFFFFFF if never), per sequence."""
    good = simulate(design, stim_seqs)
    bad = simulate(design, stim_seqs, fault)
    po = np.asarray(design.po, dtype=np.int64)
    diff = (good[:, :, po] != bad[:, :, po]).any(axis=2)   # [S][T]
    T = diff.shape[1]
    first = np.where(diff.any(axis=1), diff.argmax(axis=1), 0xFFFFFFFF)
    return first.astype(np.uint64)
