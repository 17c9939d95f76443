"""Pin the oracle's operator semantics.

Each single-operator design is simulated by the oracle's golden simulator and
compared with (a) the gate-level evaluator over every operand combination for
small widths and (b) textbook modular integer arithmetic on random 64-bit
operands.
"""
import itertools

import numpy as np
import pytest

import oracle
from bitblast import simulate
from helpers import Builder
from paper_2508_16376_amd.workloads import (ADD, AND, CONCAT, EQ, MUL, MUX, NE, NOT, OR, SHL, SHR,
                                            SLICE, SUB, ULT, XOR, counter_values)

BINARY = [ADD, SUB, AND, OR, XOR, MUL, EQ, NE, ULT, CONCAT]
UNARY = [NOT, SHL, SHR, SLICE]


def _single_op_design(op, w, in_widths, param=0):
    b = Builder()
    ins = [b.pi(x) for x in in_widths]
    n = b.node(op, w, ins, param)
    return b.design([n]), n


def _all_combinations(in_widths):
    ranges = [range(1 << x) for x in in_widths]
    return np.array(list(itertools.product(*ranges)), dtype=np.uint64)


def _oracle_vs_gates(op, w, in_widths, param=0):
    d, n = _single_op_design(op, w, in_widths, param)
    stim = _all_combinations(in_widths)          # one cycle per operand combination
    G = oracle.golden(d, stim, stim.shape[0])
    gates = simulate(d, stim[:, None, :])         # one sequence per combination
    np.testing.assert_array_equal(G[:, n], gates[:, 0, n],
                                  err_msg=f"op={op} w={w} in={in_widths} param={param}")


@pytest.mark.parametrize("op", BINARY)
def test_binary_exhaustive_small_widths(op):
    for wa, wb in itertools.product([1, 2, 3], repeat=2):
        for w in [1, 2, 3, 4]:
            if op == CONCAT and w > wa + wb:
                continue
            _oracle_vs_gates(op, w, [wa, wb])


@pytest.mark.parametrize("op", UNARY)
def test_unary_exhaustive_small_widths(op):
    for wa in [1, 2, 3, 4]:
        for w in [1, 2, 3, 4]:
            params = range(0, 6) if op != NOT else [0]
            for p in params:
                _oracle_vs_gates(op, w, [wa], p)


def test_mux_exhaustive_small_widths():
    for ws, wa, wb, w in itertools.product([1, 2], [1, 2], [1, 3], [1, 2, 3]):
        _oracle_vs_gates(MUX, w, [ws, wa, wb])


def _rand_words(k, n, w):
    v = counter_values(0xC0FFEE + k, 0, n)
    if w < 64:
        v &= np.uint64((1 << w) - 1)
    return v


PY_SEMANTICS = {
    ADD: lambda a, b, w, p: (a + b) % (1 << w),
    SUB: lambda a, b, w, p: (a - b) % (1 << w),
    AND: lambda a, b, w, p: (a & b) % (1 << w),
    OR: lambda a, b, w, p: (a | b) % (1 << w),
    XOR: lambda a, b, w, p: (a ^ b) % (1 << w),
    MUL: lambda a, b, w, p: (a * b) % (1 << w),
    EQ: lambda a, b, w, p: int(a == b),
    NE: lambda a, b, w, p: int(a != b),
    ULT: lambda a, b, w, p: int(a < b),
}


@pytest.mark.parametrize("op", list(PY_SEMANTICS))
@pytest.mark.parametrize("w", [64, 32, 17])
def test_random_wide_against_integer_arithmetic(op, w):
    wo = 1 if op in (EQ, NE, ULT) else w
    d, n = _single_op_design(op, wo, [w, w])
    n_cases = 3000
    a = _rand_words(op * 100 + w, n_cases, w)
    b = _rand_words(op * 100 + w + 7, n_cases, w)
    b[::5] = a[::5]                                   # equal operands for the compares
    stim = np.stack([a, b], axis=1)
    G = oracle.golden(d, stim, n_cases)
    expect = np.array([PY_SEMANTICS[op](int(x), int(y), wo, 0) for x, y in zip(a, b)], dtype=np.uint64)
    np.testing.assert_array_equal(G[:, n], expect)


@pytest.mark.parametrize("op", [SHL, SHR, SLICE, NOT])
def test_random_wide_unary_against_gates(op):
    for w, wa, p in [(64, 64, 0), (64, 64, 13), (64, 64, 63), (32, 64, 32), (16, 64, 48), (64, 32, 70)]:
        d, n = _single_op_design(op, w, [wa], p)
        a = _rand_words(op * 7 + p, 500, wa)[:, None]
        G = oracle.golden(d, a, a.shape[0])
        gates = simulate(d, a[:, None, :])
        np.testing.assert_array_equal(G[:, n], gates[:, 0, n])


def test_random_wide_mul_and_concat_against_gates():
    for op, w, wa, wb in [(MUL, 64, 64, 64), (MUL, 32, 32, 16), (CONCAT, 64, 32, 32), (CONCAT, 40, 24, 16)]:
        d, n = _single_op_design(op, w, [wa, wb])
        a = _rand_words(w + wa, 300, wa)
        b = _rand_words(w + wb + 1, 300, wb)
        stim = np.stack([a, b], axis=1)
        G = oracle.golden(d, stim, 300)
        gates = simulate(d, stim[:, None, :])
        np.testing.assert_array_equal(G[:, n], gates[:, 0, n])
