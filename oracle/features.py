"""Reference of the load predictor's per-fault features (test infrastructure).

For a fault (site s, bit b, stuck v) over a golden trace of T cycles:

  0  log2(1 + cone), cone = number of distinct nodes reached from s through
     combinational users, registers fed counted but not crossed, capped at
     CONE_CAP (the site itself is not counted);
  1  combinational level of s divided by the deepest level (1 if that is 0);
  2  register depth: fewest registers on any path from s to a primary output,
     capped at DEPTH_CAP; -1 when no output is reachable;
  3  log2(width of s);
  4  toggle rate of bit b of s: cycles t in 1..T-1 where it differs from
     cycle t-1, divided by max(1, T-1);
  5  excitation rate: cycles where bit b differs from v, divided by T (a bit
     flip is excited once, in its cycle t0, if t0 < T).

Plain Python graph walks and numpy over the oracle's golden trace.
"""
from __future__ import annotations

from collections import deque

import numpy as np

from paper_2508_16376_amd.workloads import ARITY, CONST, FLIP, PI, REG

CONE_CAP = 1024
DEPTH_CAP = 16
N_FEATURES = 6


def _users(design):
    N = design.num_nodes
    comb_users = [[] for _ in range(N)]
    reg_users = [[] for _ in range(N)]
    nd = design.nodes
    for n in range(N):
        op = int(nd["op"][n])
        if op == REG:
            reg_users[int(nd["in0"][n])].append(n)
        elif op not in (CONST, PI):
            for k in range(ARITY[op]):
                i = int(nd[f"in{k}"][n])
                if n not in comb_users[i]:
                    comb_users[i].append(n)
    return comb_users, reg_users


def levels(design) -> np.ndarray:
    nd = design.nodes
    N = design.num_nodes
    lvl = np.full(N, -1, dtype=np.int64)

    def level_of(root):
        stack = [root]
        while stack:
            n = stack[-1]
            if lvl[n] >= 0:
                stack.pop()
                continue
            op = int(nd["op"][n])
            if op in (CONST, PI, REG):
                lvl[n] = 0
                stack.pop()
                continue
            ins = [int(nd[f"in{k}"][n]) for k in range(ARITY[op])]
            todo = [i for i in ins if lvl[i] < 0]
            if todo:
                stack.extend(todo)
            else:
                lvl[n] = 1 + max(lvl[i] for i in ins)
                stack.pop()

    for n in range(N):
        if lvl[n] < 0:
            level_of(n)
    return lvl


def cone_size(design, site: int, comb_users=None, reg_users=None) -> int:
    if comb_users is None:
        comb_users, reg_users = _users(design)
    seen = {site}
    q = deque([site])
    count = 0
    while q and count < CONE_CAP:
        u = q.popleft()
        for c in comb_users[u]:
            if c not in seen:
                seen.add(c)
                count += 1
                q.append(c)
        for r in reg_users[u]:
            if r not in seen:
                seen.add(r)
                count += 1
    return min(count, CONE_CAP)


def register_depth(design) -> np.ndarray:
    """Fewest registers on a path from each node to a primary output (0-1 BFS
    backwards from the outputs); -1 when unreachable."""
    nd = design.nodes
    N = design.num_nodes
    INF = 1 << 30
    dist = np.full(N, INF, dtype=np.int64)
    dq = deque()
    for p in design.po:
        dist[int(p)] = 0
        dq.append(int(p))
    while dq:
        u = dq.popleft()
        op = int(nd["op"][u])
        if op == REG:
            d = int(nd["in0"][u])
            if dist[u] + 1 < dist[d]:
                dist[d] = dist[u] + 1
                dq.append(d)
        elif op not in (CONST, PI):
            for k in range(ARITY[op]):
                i = int(nd[f"in{k}"][u])
                if dist[u] < dist[i]:
                    dist[i] = dist[u]
                    dq.appendleft(i)
    return np.where(dist >= INF, -1, np.minimum(dist, DEPTH_CAP))


def features(design, G: np.ndarray, faults: np.ndarray) -> np.ndarray:
    """[F][6] float64 features (G is the oracle's golden trace [T][N])."""
    T = G.shape[0]
    comb_users, reg_users = _users(design)
    lvl = levels(design)
    maxl = max(1, int(lvl.max()))
    rdep = register_depth(design)
    out = np.zeros((faults.size, N_FEATURES), dtype=np.float64)
    cone_cache: dict[int, int] = {}
    for i, f in enumerate(faults):
        s, b, v = int(f["site"]), int(f["bit"]), int(f["stuck"])
        if s not in cone_cache:
            cone_cache[s] = cone_size(design, s, comb_users, reg_users)
        bits = ((G[:, s] >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
        toggles = int(np.count_nonzero(bits[1:] != bits[:-1]))
        excited = int(int(f["t0"]) < T) if v == FLIP else int(np.count_nonzero(bits != v))
        out[i] = [np.log2(1.0 + cone_cache[s]), lvl[s] / maxl, float(rdep[s]),
                  np.log2(float(design.nodes["width"][s])), toggles / max(1, T - 1), excited / T]
    return out
