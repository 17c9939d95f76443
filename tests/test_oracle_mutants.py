"""The pins bite: plausible mistakes planted in copies of the oracle are caught.

Each mutant is the oracle source with one textual change, compiled with gcc on
the CPU.  A battery of pin checks (operators against the gate-level evaluator,
brute force with event counts, the counter closed form) must fail on it.
"""
import itertools

import numpy as np
import pytest

import oracle
from bitblast import simulate
from helpers import Builder, all_faults, all_flip_faults, fault_tuple, faults
from paper_2508_16376_amd.workloads import (ADD, AND, CONCAT, EQ, MUL, MUX, NE, NOT, OR, SHL, SHR,
                                            SLICE, SUB, ULT, XOR)
from test_oracle_brute import reference_counts, tiny_designs

MUTANTS = {
    "mux_legs_swapped": ("r = (a != 0) ? c : b;", "r = (a != 0) ? b : c;"),
    "sub_reversed": ("case O_SUB: r = a - b;", "case O_SUB: r = b - a;"),
    "ult_is_ule": ("case O_ULT: r = (a < b);", "case O_ULT: r = (a <= b);"),
    "concat_uses_wrong_width": ("unsigned wb = all[nd->in[1]].width;", "unsigned wb = all[nd->in[0]].width;"),
    "force_polarity_swapped": ("return f->stuck ? (v | bit) : (v & ~bit);",
                               "return f->stuck ? (v & ~bit) : (v | bit);"),
    "o0_register_events_dropped": ("div_in = state[n] != g[n];", "div_in = 0;"),
    "o0_detect_late": ("if (val[d->po[i]] != g[d->po[i]] && detect == O_UNDET) detect = t;",
                       "if (val[d->po[i]] != g[d->po[i]] && detect == O_UNDET) detect = t + 1;"),
    "o1_no_register_fanout": ("s->rnext[nnext] = r;\n                    s->rnextv[nnext] = v & o_mask(d->nd[r].width);\n                    nnext++;",
                              "(void)r;"),
    "o1_output_divergence_not_counted": ("if (div_in || div_out) { ev++; words += o_event_words(x); }",
                                         "if (div_in) { ev++; words += o_event_words(x); }"),
    "o1_register_words_dropped": ("            words += 2u * o_ww(&d->nd[r]);\n", ""),
    "wide_words_not_doubled": ("return x->width > 32 ? 2u : 1u;", "return 1u;"),
    "event_words_without_operands": ("return (k + 2u) * o_ww(x);", "return 2u * o_ww(x);"),
    "shr_is_shl": ("case O_SHR: r = k >= 64 ? 0 : (a >> k);", "case O_SHR: r = k >= 64 ? 0 : (a << k);"),
    "mul_is_add": ("case O_MUL: r = a * b;", "case O_MUL: r = a + b;"),
    "flip_one_cycle_late": ("return t == f->t0 ? (v ^ bit) : v;", "return t == f->t0 + 1u ? (v ^ bit) : v;"),
    "flip_is_permanent": ("return t == f->t0 ? (v ^ bit) : v;", "return t >= f->t0 ? (v ^ bit) : v;"),
    "reset_value_ignored": ("state[r] = d->nd[r].param & o_mask(d->nd[r].width);\n    }\n    for (uint32_t t = 0; t < T; ++t) {\n        const uint64_t* row = stim + (size_t)t * d->npi;",
                            "state[r] = 0;\n    }\n    for (uint32_t t = 0; t < T; ++t) {\n        const uint64_t* row = stim + (size_t)t * d->npi;"),
}


def _ops_pass(lib) -> bool:
    for op, ws in [(ADD, [2, 3]), (SUB, [3, 2]), (AND, [2, 2]), (OR, [2, 2]), (XOR, [3, 3]),
                   (MUL, [3, 3]), (EQ, [2, 3]), (NE, [2, 2]), (ULT, [3, 2]), (CONCAT, [2, 2]),
                   (MUX, [1, 2, 2]), (NOT, [3]), (SHL, [3]), (SHR, [3]), (SLICE, [3])]:
        b = Builder()
        ins = [b.pi(x) for x in ws]
        w = 4 if op == CONCAT else 3
        n = b.node(op, w, ins, 1 if op in (SHL, SHR, SLICE) else 0)
        d = b.design([n])
        stim = np.array(list(itertools.product(*[range(1 << x) for x in ws])), dtype=np.uint64)
        G = lib.golden(d, stim, stim.shape[0])
        if not np.array_equal(G[:, n], simulate(d, stim[:, None, :])[:, 0, n]):
            return False
    return True


def _brute_pass(lib) -> bool:
    T = 4
    seqs_int = np.arange(0, 4096, 61, dtype=np.uint64)
    seqs = np.zeros((seqs_int.size, T, 2), dtype=np.uint64)
    for t in range(T):
        chunk = (seqs_int >> np.uint64(3 * t)) & np.uint64(7)
        seqs[:, t, 0] = chunk & np.uint64(1)
        seqs[:, t, 1] = chunk >> np.uint64(1)
    for d in tiny_designs():
        fl = np.concatenate([all_faults(d), all_flip_faults(d, T)])
        for drop in (True, False):
            ref = [reference_counts(d, seqs, fault_tuple(f), drop) for f in fl]
            for j in range(seqs.shape[0]):
                for variant in (0, 1):
                    det, ev = lib.fault_sim(d, seqs[j], T, fl, drop=drop, variant=variant)
                    for i in range(fl.size):
                        if det[i] != ref[i][0][j] or ev[i] != ref[i][1][j]:
                            return False
    # byte-model words and the last divergent-register cycle, on one design
    d = tiny_designs()[4]
    fl = np.concatenate([all_faults(d), all_flip_faults(d, T)])
    for drop in (True, False):
        ref = [reference_counts(d, seqs, fault_tuple(f), drop, stats=True) for f in fl]
        for j in range(seqs.shape[0]):
            for variant in (0, 1):
                _, _, words, lastreg = lib.fault_sim_stats(d, seqs[j], T, fl, drop=drop, variant=variant)
                for i in range(fl.size):
                    if words[i] != ref[i][2][j] or lastreg[i] != ref[i][3][j]:
                        return False
    return True


def _counter_pass(lib) -> bool:
    b = Builder()
    b.pi(1)
    cnt = b.reg(8)
    one = b.const(8, 1)
    add = b.node(ADD, 8, (cnt, one))
    b.set_d(cnt, add)
    d = b.design([cnt])
    T = 300
    stim = np.zeros((T, 1), dtype=np.uint64)
    G = lib.golden(d, stim, T)
    if not np.array_equal(G[:, cnt], np.arange(T, dtype=np.uint64) % np.uint64(256)):
        return False
    fl = faults([(cnt, k, 0) for k in range(8)])
    for variant in (0, 1):
        det, _ = lib.fault_sim(d, stim, T, fl, variant=variant)
        want = [2 ** k if 2 ** k < T else oracle.UNDETECTED for k in range(8)]
        if list(det) != want:
            return False
    # a 64-bit counter, SA1 on a register bit: 7 words of two halves each
    b = Builder()
    b.pi(1)
    cnt = b.reg(64)
    add = b.node(ADD, 64, (cnt, b.const(64, 1)))
    b.set_d(cnt, add)
    d = b.design([cnt])
    for variant in (0, 1):
        _, _, words, _ = lib.fault_sim_stats(d, stim[:20], 20, faults([(cnt, 5, 1)]), variant=variant)
        if int(words[0]) != 14:
            return False
    return True


def _battery(lib) -> bool:
    return _ops_pass(lib) and _counter_pass(lib) and _brute_pass(lib)


def test_unmodified_source_passes_battery(tmp_path):
    lib = oracle.compile_variant(oracle.source_text(), str(tmp_path), "clean")
    assert _battery(lib)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    lib = oracle.compile_variant(src.replace(old, new), str(tmp_path), name)
    assert not _battery(lib), f"planted mistake {name} was not caught"
