"""The C-ABI library loads, exports every symbol the header declares, and its
host-side validation rejects malformed designs (no GPU needed: validation runs
before any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from helpers import Builder
from paper_2508_16376_amd import riros
from paper_2508_16376_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "riros.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\*\s]+?\b(riros_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ["riros_load_design", "riros_golden_sim", "riros_fault_sim"]:
        assert name in fns


def test_library_exports_every_declared_symbol():
    L = riros.lib()
    for name in header_functions():
        assert hasattr(L, name), name
    assert set(riros.EXPORTED) == set(header_functions())


def _load(design):
    nodes = np.ascontiguousarray(design.nodes)
    po = np.ascontiguousarray(design.po, dtype=np.uint32)
    desc = riros._DesignDesc(nodes.size, riros._ptr(nodes), design.num_pi, po.size, riros._ptr(po))
    h = ctypes.c_void_p()
    rc = riros.lib().riros_load_design(ctypes.byref(desc), ctypes.byref(h))
    if rc == 0:
        riros.lib().riros_free_design(h)
    return rc, riros.lib().riros_last_error().decode()


def test_combinational_loop_rejected():
    b = Builder()
    a = b.pi(4)
    x = b.node(W.ADD, 4, (a, 0))
    y = b.node(W.XOR, 4, (x, a))
    b.rows[x] = (W.ADD, 4, 0, a, y, 0, 0)        # x reads y, y reads x
    rc, msg = _load(b.design([y]))
    assert rc == riros.RIROS_ECYCLE, msg


@pytest.mark.parametrize("case", ["width0", "width65", "badop", "badin", "badpi", "badpo", "regwidth"])
def test_malformed_design_rejected(case):
    b = Builder()
    a = b.pi(8)
    r = b.reg(8)
    x = b.node(W.ADD, 8, (a, r))
    b.set_d(r, x)
    d = b.design([x])
    n = d.nodes
    if case == "width0":
        n["width"][x] = 0
    elif case == "width65":
        n["width"][x] = 65
    elif case == "badop":
        n["op"][x] = 99
    elif case == "badin":
        n["in1"][x] = 1000
    elif case == "badpi":
        n["param"][a] = 5
    elif case == "badpo":
        d.po[0] = 77
    elif case == "regwidth":
        n["width"][r] = 4
    rc, msg = _load(d)
    assert rc == riros.RIROS_EINVAL, (case, rc, msg)
    assert msg


def test_mode_constants_match_the_header():
    text = open(os.path.join(ROOT, "include", "riros.h")).read()
    modes = {m: int(v) for m, v in re.findall(r"#define RIROS_MODE_(\w+) (\d+)", text)}
    assert modes == {"PLAIN": riros.MODE_PLAIN, "TWO_D": riros.MODE_TWO_D, "CONCURRENT": riros.MODE_CONCURRENT}
