"""Seeded synthetic workloads: word-level RTL designs, stimuli and fault lists.

This module only draws structure and random numbers.  It evaluates no node
and simulates nothing, so both the HIP path and the CPU oracle can take its
output as plain inputs.

A design is a flat node list (numpy structured array, 24 bytes per node, the
layout of ``riros_node`` in the C header) plus a primary-output list and a
primary-input count.  Node fields:

    op, width      operator code and result width in bits (1..64)
    in0, in1, in2  operand node ids (unused ones are 0)
    param          CONST value, PI stimulus column, REG reset value,
                   constant shift amount, or SLICE low bit

Register D inputs are ``in0`` of a REG node; registers break every cycle, so
the combinational part is acyclic.  The paper compiles RTL into such a graph of
RTL nodes (Sec. II-B) and injects stuck-at faults on wires and registers
(Sec. IV-A, Sec. V-A); the designs themselves are not published, so seeded
layered DAGs and seeded templates of the same shape stand in for them.

Random numbers come from a counter-based generator: value ``c`` of stream
``s`` is the SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014) of
``s + (c + 1) * 0x9E3779B97F4A7C15``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Operator codes: the values of the RIROS_OP_* constants of the C interface.
CONST, PI, REG, ADD, SUB, AND, OR, XOR, NOT, MUX, SHL, SHR, EQ, NE, ULT, SLICE, CONCAT, MUL = range(18)
OP_NAMES = ["CONST", "PI", "REG", "ADD", "SUB", "AND", "OR", "XOR", "NOT", "MUX",
            "SHL", "SHR", "EQ", "NE", "ULT", "SLICE", "CONCAT", "MUL"]
# Number of operand slots each op reads (REG reads in0 as its D input).
ARITY = {CONST: 0, PI: 0, REG: 1, ADD: 2, SUB: 2, AND: 2, OR: 2, XOR: 2, NOT: 1,
         MUX: 3, SHL: 1, SHR: 1, EQ: 2, NE: 2, ULT: 2, SLICE: 1, CONCAT: 2, MUL: 2}

NODE_DTYPE = np.dtype([("op", "u1"), ("width", "u1"), ("pad", "<u2"),
                       ("in0", "<u4"), ("in1", "<u4"), ("in2", "<u4"),
                       ("param", "<u8")])
# stuck: 0 or 1 for a stuck-at fault; FLIP for a single bit flip in cycle t0.
FAULT_DTYPE = np.dtype([("site", "<u4"), ("bit", "u1"), ("stuck", "u1"), ("t0", "<u2")])
FLIP = 2
assert NODE_DTYPE.itemsize == 24 and FAULT_DTYPE.itemsize == 8

UNDETECTED = 0xFFFFFFFF
MASTER_SEED = 2508163760

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_U64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser applied elementwise to a uint64 array."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def counter_values(seed: int, start: int, n: int) -> np.ndarray:
    """Values ``start .. start+n-1`` of the counter-based stream ``seed``."""
    ctr = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = np.uint64(seed & _U64) + ctr * _GAMMA
    return splitmix64(x)


def sub_seed(seed: int, k: int) -> int:
    return int(counter_values(seed, k - 1, 1)[0])


class Stream:
    """Sequential reader over one counter-based stream, drawn in blocks."""

    def __init__(self, seed: int, block: int = 1 << 16):
        self.seed = seed & _U64
        self.ctr = 0
        self.block = block
        self._buf = np.empty(0, dtype=np.uint64)
        self._pos = 0

    def _refill(self):
        self._buf = counter_values(self.seed, self.ctr, self.block)
        self.ctr += self.block
        self._pos = 0

    def u64(self) -> int:
        if self._pos >= self._buf.size:
            self._refill()
        v = int(self._buf[self._pos])
        self._pos += 1
        return v

    def uniform(self) -> float:
        return (self.u64() >> 11) * (1.0 / (1 << 53))

    def below(self, m: int) -> int:
        """Uniform integer in [0, m)."""
        return min(int(self.uniform() * m), m - 1)

    def choice(self, weights) -> int:
        u = self.uniform() * sum(weights)
        acc = 0.0
        for i, w in enumerate(weights):
            acc += w
            if u < acc:
                return i
        return len(weights) - 1

    def many(self, n: int) -> np.ndarray:
        out = np.empty(n, dtype=np.uint64)
        got = 0
        while got < n:
            if self._pos >= self._buf.size:
                self._refill()
            take = min(n - got, self._buf.size - self._pos)
            out[got:got + take] = self._buf[self._pos:self._pos + take]
            self._pos += take
            got += take
        return out


@dataclass
class Design:
    nodes: np.ndarray            # NODE_DTYPE[N]
    po: np.ndarray               # uint32[num_po]
    num_pi: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def num_nodes(self) -> int:
        return int(self.nodes.size)


def mask_of(w: int) -> int:
    return _U64 if w >= 64 else (1 << w) - 1


# ---------------------------------------------------------------------------
# Layered random DAG (the shape of the small and medium configurations)
# ---------------------------------------------------------------------------

# Operator categories and their weights (ADD/SUB 20, AND/OR/XOR 15, MUX 15,
# constant shift 10, compare 10, slice/concat 10, MUL low half 5), normalised
# over the operator nodes; registers are counted separately.
OP_MIX = [((ADD, SUB), 20), ((AND, OR, XOR), 15), ((MUX,), 15), ((SHL, SHR), 10),
          ((EQ, NE, ULT), 10), ((SLICE, CONCAT), 10), ((MUL,), 5)]


class _Pools:
    """Per-width node pools, in creation order, for operand selection."""

    def __init__(self):
        self.by_w: dict[int, list[int]] = {}
        self.level_start: dict[int, list[int]] = {}   # width -> list index where each level starts
        self.unused: dict[int, list[int]] = {}        # width -> nodes without fan-out yet

    def add(self, nid: int, w: int):
        self.by_w.setdefault(w, []).append(nid)
        self.unused.setdefault(w, []).append(nid)


def gen_layered(seed: int, *, n_nodes: int, n_regs: int, n_pi: int, n_po: int,
                n_levels: int, widths, wweights, name: str = "layered",
                max_mul_w: int = 32, fresh_bias: float = 0.7) -> Design:
    """Random levelised word-level design.

    ``n_nodes`` counts every node (PIs, registers and operators).  Operators get
    a target level in 1..n_levels; operand 0 comes from the level just below,
    so the combinational depth is ``n_levels``.  Operands prefer nodes that have
    no fan-out yet, so little logic is left dangling.  Register widths follow
    ``wweights``; each register's D input is an operator of the same width.
    """
    st = Stream(sub_seed(seed, 1))
    n_ops = n_nodes - n_pi - n_regs
    assert n_ops >= n_levels >= 1
    widths = list(widths)
    wweights = list(wweights)

    ops_cat = [c for c, _ in OP_MIX]
    ops_w = [w for _, w in OP_MIX]

    node_op = []
    node_w = []
    node_in = []
    node_param = []
    node_level = []
    fanout = []

    def new(op, w, ins, param, level):
        nid = len(node_op)
        node_op.append(op)
        node_w.append(w)
        node_in.append(list(ins) + [0] * (3 - len(ins)))
        node_param.append(param)
        node_level.append(level)
        fanout.append(0)
        return nid

    # Level 0: primary inputs and registers.
    pools = _Pools()
    level_nodes = {0: []}
    for i in range(n_pi):
        w = widths[st.choice(wweights)]
        nid = new(PI, w, [], i, 0)
        level_nodes[0].append(nid)
    reg_ids = []
    for _ in range(n_regs):
        w = widths[st.choice(wweights)]
        nid = new(REG, w, [0], 0, 0)
        reg_ids.append(nid)
        level_nodes[0].append(nid)

    # Target levels for operators: every level gets at least one operator.
    lv = [1 + (i % n_levels) if i < n_levels else 1 + st.below(n_levels) for i in range(n_ops)]
    lv.sort()

    # Per-level, per-width node lists for operand selection.
    below = {}          # width -> list of node ids at levels < current level
    below_any = []
    by_level_w = {}     # (level, width) -> ids
    for nid in level_nodes[0]:
        below.setdefault(node_w[nid], []).append(nid)
        below_any.append(nid)
        by_level_w.setdefault((0, node_w[nid]), []).append(nid)
    unused = {}         # width -> set-like list of ids with no fan-out (levels < current)
    unused_pos = {}     # id -> position in its unused list (for O(1) removal)

    def unused_add(nid):
        lst = unused.setdefault(node_w[nid], [])
        unused_pos[nid] = len(lst)
        lst.append(nid)

    def unused_remove(nid):
        if nid not in unused_pos:
            return
        lst = unused[node_w[nid]]
        p = unused_pos.pop(nid)
        last = lst.pop()
        if last != nid:
            lst[p] = last
            unused_pos[last] = p

    for nid in level_nodes[0]:
        if node_op[nid] != PI or True:
            unused_add(nid)

    def use(nid):
        fanout[nid] += 1
        unused_remove(nid)
        return nid

    def pick_w(w, fresh=True):
        """An operand of width w from lower levels (fresh nodes first)."""
        if fresh and st.uniform() < fresh_bias:
            lst = unused.get(w)
            if lst:
                return use(lst[st.below(len(lst))])
        lst = below.get(w)
        if lst:
            return use(lst[st.below(len(lst))])
        return use(below_any[st.below(len(below_any))])

    def pick_prev(level, w):
        lst = by_level_w.get((level - 1, w))
        if lst:
            return use(lst[st.below(len(lst))])
        cands = [x for x in level_nodes.get(level - 1, [])]
        if cands:
            return use(cands[st.below(len(cands))])
        return pick_w(w)

    cur_level = 1
    pending = []   # nodes created at cur_level, published to "below" when the level ends

    def publish():
        for nid in pending:
            below.setdefault(node_w[nid], []).append(nid)
            below_any.append(nid)
            unused_add(nid)

    for l in lv:
        if l != cur_level:
            publish()
            pending = []
            cur_level = l
        cat = ops_cat[st.choice(ops_w)]
        op = cat[st.below(len(cat))]
        w = widths[st.choice(wweights)]
        if op in (SHL, SHR) and w < 8:
            w = 8 if 8 in widths else max(widths)
        if op == MUL:
            w = min(w, max_mul_w)
        if op == SLICE and w >= max(widths):
            w = max(x for x in widths if x < max(widths))
        if op == CONCAT and w < 16:
            op = SLICE
        if op in (EQ, NE, ULT):
            wc = widths[st.choice(wweights)]
            a = pick_prev(l, wc)
            b = pick_w(wc)
            nid = new(op, 1, [a, b], 0, l)
        elif op == MUX:
            sel = pick_prev(l, 1)
            a = pick_w(w)
            b = pick_w(w)
            nid = new(op, w, [sel, a, b], 0, l)
        elif op in (SHL, SHR):
            a = pick_prev(l, w)
            k = 1 + st.below(max(1, w - 1))
            nid = new(op, w, [a], k, l)
        elif op == SLICE:
            wider = [x for x in widths if x > w]
            wa = wider[st.below(len(wider))]
            a = pick_prev(l, wa)
            wa_real = node_w[a]
            lo = st.below(max(1, wa_real - w + 1)) if wa_real > w else 0
            nid = new(op, w, [a], lo, l)
        elif op == CONCAT:
            half = w // 2
            a = pick_prev(l, half)
            b = pick_w(half)
            wsum = min(64, node_w[a] + node_w[b])
            nid = new(op, wsum, [a, b], 0, l)
        else:   # ADD SUB AND OR XOR MUL
            a = pick_prev(l, w)
            b = pick_w(w)
            nid = new(op, w, [a, b], 0, l)
        pending.append(nid)
        by_level_w.setdefault((l, node_w[nid]), []).append(nid)
        level_nodes.setdefault(l, []).append(nid)
    publish()

    # Register D inputs: an operator of the register's width, dangling ones first.
    ops_by_w = {}
    for nid in range(len(node_op)):
        if node_op[nid] not in (PI, REG):
            ops_by_w.setdefault(node_w[nid], []).append(nid)
    for r in reg_ids:
        w = node_w[r]
        if w not in ops_by_w:
            w = max(ops_by_w, key=lambda x: len(ops_by_w[x]))
            node_w[r] = w
        lst = unused.get(w)
        fresh_ops = [x for x in (lst or []) if node_op[x] not in (PI, REG)]
        if fresh_ops:
            d = fresh_ops[st.below(len(fresh_ops))]
        else:
            d = ops_by_w[w][st.below(len(ops_by_w[w]))]
        node_in[r][0] = use(d)

    # Primary outputs: dangling operators of the deepest levels first.
    dangling = [nid for nid in range(len(node_op))
                if fanout[nid] == 0 and node_op[nid] not in (PI, REG)]
    dangling.sort(key=lambda x: (-node_level[x], x))
    po = dangling[:n_po]
    if len(po) < n_po:
        rest = [nid for nid in range(len(node_op)) if node_op[nid] not in (PI, REG) and nid not in set(po)]
        rest.sort(key=lambda x: (-node_level[x], x))
        po += rest[:n_po - len(po)]

    nodes = np.zeros(len(node_op), dtype=NODE_DTYPE)
    nodes["op"] = node_op
    nodes["width"] = node_w
    ins = np.asarray(node_in, dtype=np.uint32)
    nodes["in0"] = ins[:, 0]
    nodes["in1"] = ins[:, 1]
    nodes["in2"] = ins[:, 2]
    nodes["param"] = np.asarray(node_param, dtype=np.uint64)
    meta = {"levels": n_levels, "n_regs": n_regs,
            "dangling": int(sum(1 for nid in range(len(node_op))
                                if fanout[nid] == 0 and nid not in set(po)
                                and node_op[nid] != PI))}
    return Design(nodes, np.asarray(po, dtype=np.uint32), n_pi, name, meta)


# ---------------------------------------------------------------------------
# Template designs (the heavy-tailed configurations)
# ---------------------------------------------------------------------------

class _Net:
    """Append-only node list for template construction."""

    def __init__(self):
        self.op, self.w, self.ins, self.param = [], [], [], []

    def add(self, op, w, ins=(), param=0):
        self.op.append(op)
        self.w.append(w)
        self.ins.append(list(ins) + [0] * (3 - len(ins)))
        self.param.append(param)
        return len(self.op) - 1

    def set_in0(self, n, x):
        self.ins[n][0] = x

    def design(self, po, num_pi, name, meta):
        nodes = np.zeros(len(self.op), dtype=NODE_DTYPE)
        nodes["op"] = self.op
        nodes["width"] = self.w
        ins = np.asarray(self.ins, dtype=np.uint32)
        nodes["in0"], nodes["in1"], nodes["in2"] = ins[:, 0], ins[:, 1], ins[:, 2]
        nodes["param"] = np.asarray(self.param, dtype=np.uint64)
        return Design(nodes, np.asarray(po, dtype=np.uint32), num_pi, name, meta)


def gen_templates(seed: int, *, n_nodes: int, n_pi: int = 128, acc_share: float = 0.02,
                  name: str = "templates") -> Design:
    """Design assembled from seeded templates sharing the primary inputs:

      pipelined datapath  k = 2..4 register stages of width 8/16/32; the first
                          stage takes the XOR of two input slices (masked by
                          a constant AND in some pipelines, before any
                          register, so a masked bit never reaches state); each
                          stage mixes its register with an input slice
                          (ADD/XOR/SUB), some stages choosing by an input
                          compare between two such updates; the last stage is
                          an output, so a divergence reaches it within k
                          cycles of its excitation;
      FSM                 8-bit state, next state chosen by an input bit
                          between two update rules; the state, mixed with an
                          input, is an output;
      accumulator         32-bit acc <- acc + (a ^ b) observed only through
                          acc == constant; a divergence stays in the state for
                          the whole run without reaching an output.

    Accumulators are added until they hold about ``acc_share`` of the bits
    that can carry a fault, so about that share of a uniform fault list stays
    latent in state, and nearly all other faults are detected, or leave no
    divergent state, within ten cycles.
    """
    st = Stream(sub_seed(seed, 1))
    net = _Net()
    pis = []
    for i in range(n_pi):
        pis.append(net.add(PI, 32, (), i))
    po = []
    acc_bits = 0
    all_bits = 0

    def count(n):
        nonlocal all_bits
        all_bits += net.w[n]
        return n

    def pi_slice(w):
        p = pis[st.below(n_pi)]
        if w == 32:
            return p
        return count(net.add(SLICE, w, (p,), st.below(33 - w)))

    while len(net.op) < n_nodes:
        want_acc = acc_bits < acc_share * max(all_bits, 1)
        kind = 2 if want_acc else (0 if st.uniform() < 0.8 else 1)
        if kind == 0:
            # pipelined datapath
            w = (8, 16, 32)[st.below(3)]
            k = 2 + st.below(3)
            v = count(net.add(XOR, w, (pi_slice(w), pi_slice(w))))
            if st.uniform() < 0.15:
                m = net.add(CONST, w, (), int(st.u64() & mask_of(w)))
                v = count(net.add(AND, w, (v, m)))
            for _ in range(k):
                r = count(net.add(REG, w, (v,), 0))
                op = (ADD, XOR, SUB, ADD, XOR)[st.below(5)]
                v = count(net.add(op, w, (r, pi_slice(w))))
                if st.uniform() < 0.08:
                    sel = count(net.add(ULT, 1, (pi_slice(8), net.add(CONST, 8, (), 128))))
                    alt = count(net.add(XOR, w, (r, pi_slice(w))))
                    v = count(net.add(MUX, w, (sel, v, alt)))
            po.append(v)
        elif kind == 1:
            # FSM with 8-bit state
            s = count(net.add(REG, 8, (0,), 0))
            cond = count(net.add(EQ, 1, (pi_slice(1), net.add(CONST, 1, (), st.below(2)))))
            a = count(net.add(ADD, 8, (s, net.add(CONST, 8, (), 1 + st.below(255)))))
            b = count(net.add(XOR, 8, (s, pi_slice(8))))
            nxt = count(net.add(MUX, 8, (cond, a, b)))
            net.set_in0(s, nxt)
            po.append(count(net.add(XOR, 8, (s, pi_slice(8)))))
        else:
            # accumulator observed through a compare
            acc = count(net.add(REG, 32, (0,), 0))
            fx = count(net.add(XOR, 32, (pis[st.below(n_pi)], pis[st.below(n_pi)])))
            s2 = count(net.add(ADD, 32, (acc, fx)))
            net.set_in0(acc, s2)
            k = net.add(CONST, 32, (), int(st.u64() & 0xFFFFFFFF))
            po.append(count(net.add(EQ, 1, (acc, k))))
            acc_bits += 97
    meta = {"acc_share": acc_share, "acc_bits": acc_bits, "fault_bits": all_bits}
    return net.design(po, n_pi, name, meta)


# ---------------------------------------------------------------------------
# Stimulus and fault lists
# ---------------------------------------------------------------------------

def pi_widths(d: Design) -> np.ndarray:
    w = np.zeros(d.num_pi, dtype=np.int64)
    sel = d.nodes["op"] == PI
    w[d.nodes["param"][sel].astype(np.int64)] = d.nodes["width"][sel]
    return w


def gen_stimulus(seed: int, d: Design, T: int) -> np.ndarray:
    """uint64[T][num_pi]: uniform random bits per input, masked to the PI width."""
    stream = sub_seed(seed, 2)
    raw = counter_values(stream, 0, T * d.num_pi).reshape(T, d.num_pi)
    w = pi_widths(d)
    masks = np.array([mask_of(int(x)) if x > 0 else _U64 for x in w], dtype=np.uint64)
    return raw & masks[None, :]


def fault_universe(d: Design) -> tuple[np.ndarray, np.ndarray]:
    """Sites eligible for faults (operator and register nodes) and their widths."""
    ops = d.nodes["op"]
    sites = np.nonzero((ops != PI) & (ops != CONST))[0].astype(np.int64)
    return sites, d.nodes["width"][sites].astype(np.int64)


def gen_faults(seed: int, d: Design, F: int) -> np.ndarray:
    """F distinct single-bit stuck-at faults, uniform over (node bit, polarity)
    of operator and register bits, drawn without replacement."""
    sites, w = fault_universe(d)
    cum = np.concatenate([[0], np.cumsum(2 * w)])
    U = int(cum[-1])
    if F > U:
        raise ValueError(f"{F} faults requested but the universe has {U}")
    st = Stream(sub_seed(seed, 3))
    chosen = np.empty(0, dtype=np.int64)
    seen = np.zeros(0, dtype=np.int64)
    while chosen.size < F:
        need = F - chosen.size
        draw = (st.many(int(need * 1.3) + 16) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
        idx = np.minimum((draw * U).astype(np.int64), U - 1)
        # keep the first occurrence of each index, in draw order
        _, first = np.unique(idx, return_index=True)
        idx = idx[np.sort(first)]
        if seen.size:
            idx = idx[~np.isin(idx, seen)]
        idx = idx[:need]
        chosen = np.concatenate([chosen, idx])
        seen = np.sort(chosen)
    k = np.searchsorted(cum, chosen, side="right") - 1
    off = chosen - cum[k]
    out = np.zeros(F, dtype=FAULT_DTYPE)
    out["site"] = sites[k]
    out["bit"] = off // 2
    out["stuck"] = off % 2
    return out


# ---------------------------------------------------------------------------
# Initial weights of the load predictor (an input of training)
# ---------------------------------------------------------------------------

MLP_SHAPES = [(64, 6), (64,), (64, 64), (64,), (64,), (1,)]   # W1 b1 W2 b2 W3 b3


def mlp_init_weights(seed: int) -> np.ndarray:
    """He-uniform initial weights (zero biases) for the 6-64-64-1 predictor, as
    one float32 vector W1, b1, W2, b2, W3, b3 drawn from counter stream ``seed``."""
    parts = []
    ctr = 0
    fan_in = {0: 6, 2: 64, 4: 64}
    for k, shp in enumerate(MLP_SHAPES):
        n = int(np.prod(shp))
        if k in fan_in:
            u = (counter_values(seed, ctr, n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
            ctr += n
            parts.append((2.0 * u - 1.0) * np.sqrt(6.0 / fan_in[k]))
        else:
            parts.append(np.zeros(n))
    return np.concatenate(parts).astype(np.float32)


def gen_flip_faults(seed: int, d: Design, F: int, T: int) -> np.ndarray:
    """F single bit flips: site bits uniform over operator and register bits
    (with replacement), flip cycles uniform in [0, min(T, 65536))."""
    sites, w = fault_universe(d)
    cum = np.concatenate([[0], np.cumsum(w)])
    U = int(cum[-1])
    st = Stream(sub_seed(seed, 4))
    u = (st.many(F) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))
    idx = np.minimum((u * U).astype(np.int64), U - 1)
    k = np.searchsorted(cum, idx, side="right") - 1
    out = np.zeros(F, dtype=FAULT_DTYPE)
    out["site"] = sites[k]
    out["bit"] = idx - cum[k]
    out["stuck"] = FLIP
    out["t0"] = (st.many(F) % np.uint64(min(T, 65536))).astype(np.uint16)
    return out


# ---------------------------------------------------------------------------
# The named workloads
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    design: Design
    stimulus: np.ndarray
    faults: np.ndarray
    T: int


def config_seed(k: int) -> int:
    return MASTER_SEED + k


def tiny(seed: int | None = None, F: int = 2000, T: int = 128) -> Workload:
    """Tiny DAG: 120 operators + 16 registers, widths {1,8,16,32}, 8 PI, 4 PO,
    128 cycles, 2,000 stuck-at faults."""
    s = config_seed(0) if seed is None else seed
    d = gen_layered(s, n_nodes=8 + 16 + 120, n_regs=16, n_pi=8, n_po=4, n_levels=10,
                    widths=[1, 8, 16, 32], wweights=[1, 1, 1, 1], name="tiny")
    return Workload("tiny", d, gen_stimulus(s, d, T), gen_faults(s, d, F), T)


def heavy_tailed(seed: int | None = None, F: int = 200000, T: int = 5000, n_nodes: int = 100000) -> Workload:
    """Template design of 100,000 nodes (pipelines, FSMs, latent accumulators),
    5,000 cycles, 200,000 stuck-at faults."""
    s = config_seed(2) if seed is None else seed
    d = gen_templates(s, n_nodes=n_nodes, name="heavy_tailed")
    return Workload("heavy_tailed", d, gen_stimulus(s, d, T), gen_faults(s, d, F), T)


def large(seed: int | None = None, F: int = 1000000, T: int = 10000, n_nodes: int = 200000) -> Workload:
    """Template design of 200,000 nodes, 10,000 cycles, 1,000,000 stuck-at faults."""
    s = config_seed(4) if seed is None else seed
    d = gen_templates(s, n_nodes=n_nodes, name="large")
    return Workload("large", d, gen_stimulus(s, d, T), gen_faults(s, d, F), T)


def campaign(seed: int | None = None, n: int = 64, nodes=(1000, 50000), faults=(1000, 100000),
             cycles=(500, 5000), only=None) -> list[Workload]:
    """Batched campaign: n independent layered designs with node counts
    log-uniform in ``nodes``, register fraction uniform in 3..10 %, fault
    counts log-uniform in ``faults`` and cycle counts uniform in ``cycles``.
    Design k is seeded with the campaign seed + 1000 (k + 1).  ``only``: build
    just these design indexes (the others' sizes are still drawn, so design k
    is the same either way)."""
    s = config_seed(3) if seed is None else seed
    st = Stream(sub_seed(s, 7))
    out = []
    for k in range(n):
        sk = s + 1000 * (k + 1)
        N = int(round(math.exp(math.log(nodes[0]) + st.uniform() * (math.log(nodes[1]) - math.log(nodes[0])))))
        rf = 0.03 + 0.07 * st.uniform()
        F = int(round(math.exp(math.log(faults[0]) + st.uniform() * (math.log(faults[1]) - math.log(faults[0])))))
        T = cycles[0] + st.below(cycles[1] - cycles[0] + 1)
        if only is not None and k not in only:
            continue
        n_pi = min(128, max(8, N // 300))
        d = gen_layered(sk, n_nodes=N, n_regs=max(1, int(rf * N)), n_pi=n_pi, n_po=max(1, n_pi // 2),
                        n_levels=min(40, max(4, N // 100)), widths=[1, 8, 16, 32, 64], wweights=[2, 3, 2, 2, 1],
                        name=f"campaign{k}")
        U = 2 * int(fault_universe(d)[1].sum())
        out.append(Workload(f"campaign{k}", d, gen_stimulus(sk, d, T), gen_faults(sk, d, min(F, U)), T))
    return out


def medium(seed: int | None = None, F: int = 50000, T: int = 1000, n_nodes: int = 20000) -> Workload:
    """Medium DAG: 20,000 nodes over 40 levels, 512 registers, widths
    {1,8,16,32,64} weighted 2:3:2:2:1, 64 PI, 32 PO, 1,000 cycles, 50,000 faults."""
    s = config_seed(1) if seed is None else seed
    d = gen_layered(s, n_nodes=n_nodes, n_regs=512 * n_nodes // 20000, n_pi=64, n_po=32,
                    n_levels=40, widths=[1, 8, 16, 32, 64], wweights=[2, 3, 2, 2, 1],
                    name="medium")
    return Workload("medium", d, gen_stimulus(s, d, T), gen_faults(s, d, F), T)
