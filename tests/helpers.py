"""Small design builder and shared fixtures for the tests."""
from __future__ import annotations

import numpy as np

from paper_2508_16376_amd.workloads import NODE_DTYPE, FAULT_DTYPE, FLIP, PI, REG, CONST, Design


class Builder:
    """Append-only node list; returns node ids."""

    def __init__(self):
        self.rows = []
        self.num_pi = 0

    def node(self, op, width, ins=(), param=0):
        ins = list(ins) + [0] * (3 - len(ins))
        self.rows.append((op, width, 0, ins[0], ins[1], ins[2], param))
        return len(self.rows) - 1

    def pi(self, width):
        nid = self.node(PI, width, (), self.num_pi)
        self.num_pi += 1
        return nid

    def const(self, width, value):
        return self.node(CONST, width, (), value)

    def reg(self, width, init=0):
        return self.node(REG, width, (0,), init)

    def set_d(self, reg, d):
        r = list(self.rows[reg])
        r[3] = d
        self.rows[reg] = tuple(r)

    def design(self, po, name="built"):
        nodes = np.array(self.rows, dtype=NODE_DTYPE)
        return Design(nodes, np.asarray(po, dtype=np.uint32), self.num_pi, name)


def faults(rows):
    """Rows (site, bit, stuck) or (site, bit, FLIP, t0)."""
    out = np.zeros(len(rows), dtype=FAULT_DTYPE)
    for i, r in enumerate(rows):
        out[i] = (r[0], r[1], r[2], r[3] if len(r) > 3 else 0)
    return out


def fault_tuple(f):
    return (int(f["site"]), int(f["bit"]), int(f["stuck"]), int(f["t0"]))


def all_faults(design, sites=None):
    """Every (site, bit, polarity) over the given sites (default: every node)."""
    rows = []
    sites = range(design.num_nodes) if sites is None else sites
    for n in sites:
        for b in range(int(design.nodes["width"][n])):
            rows.append((n, b, 0))
            rows.append((n, b, 1))
    return faults(rows)


def all_flip_faults(design, T, sites=None):
    """A bit flip on every bit of the given sites (default: every node) in every cycle t0 < T."""
    rows = []
    sites = range(design.num_nodes) if sites is None else sites
    for n in sites:
        for b in range(int(design.nodes["width"][n])):
            for t0 in range(T):
                rows.append((n, b, FLIP, t0))
    return faults(rows)


def permute_design(design, perm):
    """Renumber nodes: new id of old node i is perm[i]."""
    perm = np.asarray(perm, dtype=np.int64)
    nodes = np.empty_like(design.nodes)
    nodes[perm] = design.nodes
    for k in ("in0", "in1", "in2"):
        nodes[k] = perm[nodes[k].astype(np.int64)]
    return Design(nodes, perm[design.po.astype(np.int64)].astype(np.uint32), design.num_pi,
                  design.name + "-perm")
