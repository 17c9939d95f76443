"""CPU oracle for RTL stuck-at fault simulation (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path (the HIP library and its binding) never
does.  ``riros_oracle.c`` holds the simulator (golden trace, O0 = every node
every cycle, O1 = only nodes with a divergent input); ``mlp.py`` holds the
float64 reference of the load predictor's network; ``features.py`` the
reference of the per-fault predictor features.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "riros_oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUT_DIR, "libriros_oracle.so")
_lib = None

UNDETECTED = 0xFFFFFFFF


def _compile(src: str, out: str, extra=()) -> str:
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread",
                    *extra, src, "-o", tmp], check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/_build/libriros_oracle.so."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        _compile(_SRC, _LIB_PATH)
    return _LIB_PATH


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


class OracleLib:
    """One compiled oracle library (the default build, or a copy compiled from
    modified source by the mutation test)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        U = ctypes.c_uint32
        lib.oracle_golden.argtypes = [P, U, P, U, U, P, U, P]
        lib.oracle_golden.restype = ctypes.c_int
        lib.oracle_fault_sim.argtypes = [ctypes.c_int, P, U, P, U, U, P, U, P, P, U,
                                         ctypes.c_int, ctypes.c_int, P, P]
        lib.oracle_fault_sim.restype = ctypes.c_int
        lib.oracle_fault_sim_ex.argtypes = [ctypes.c_int, P, U, P, U, U, P, U, P, P, U,
                                            ctypes.c_int, ctypes.c_int, P, P, P, P]
        lib.oracle_fault_sim_ex.restype = ctypes.c_int
        self.lib = lib

    def golden(self, design, stimulus: np.ndarray, T: int) -> np.ndarray:
        nodes = np.ascontiguousarray(design.nodes)
        po = np.ascontiguousarray(design.po, dtype=np.uint32)
        stim = np.ascontiguousarray(stimulus[:T], dtype=np.uint64)
        G = np.empty((T, nodes.size), dtype=np.uint64)
        rc = self.lib.oracle_golden(_ptr(nodes), nodes.size, _ptr(po), po.size, design.num_pi,
                                    _ptr(stim), T, _ptr(G))
        if rc:
            raise ValueError(f"oracle_golden failed with {rc}")
        return G

    def fault_sim(self, design, stimulus, T, faults, *, G=None, drop=True, variant=1, nthreads=None):
        if G is None:
            G = self.golden(design, stimulus, T)
        nodes = np.ascontiguousarray(design.nodes)
        po = np.ascontiguousarray(design.po, dtype=np.uint32)
        stim = np.ascontiguousarray(stimulus[:T], dtype=np.uint64)
        G = np.ascontiguousarray(G[:T], dtype=np.uint64)
        fl = np.ascontiguousarray(faults)
        F = fl.size
        detect = np.empty(F, dtype=np.uint32)
        events = np.empty(F, dtype=np.uint64)
        nt = default_threads() if nthreads is None else nthreads
        rc = self.lib.oracle_fault_sim(variant, _ptr(nodes), nodes.size, _ptr(po), po.size,
                                       design.num_pi, _ptr(stim), T, _ptr(G), _ptr(fl), F,
                                       1 if drop else 0, nt, _ptr(detect), _ptr(events))
        if rc:
            raise ValueError(f"oracle_fault_sim failed with {rc}")
        return detect, events

    def fault_sim_stats(self, design, stimulus, T, faults, *, G=None, drop=True, variant=1, nthreads=None):
        if G is None:
            G = self.golden(design, stimulus, T)
        nodes = np.ascontiguousarray(design.nodes)
        po = np.ascontiguousarray(design.po, dtype=np.uint32)
        stim = np.ascontiguousarray(stimulus[:T], dtype=np.uint64)
        G = np.ascontiguousarray(G[:T], dtype=np.uint64)
        fl = np.ascontiguousarray(faults)
        F = fl.size
        detect = np.empty(F, dtype=np.uint32)
        events = np.empty(F, dtype=np.uint64)
        words = np.empty(F, dtype=np.uint64)
        lastreg = np.empty(F, dtype=np.uint32)
        nt = default_threads() if nthreads is None else nthreads
        rc = self.lib.oracle_fault_sim_ex(variant, _ptr(nodes), nodes.size, _ptr(po), po.size,
                                          design.num_pi, _ptr(stim), T, _ptr(G), _ptr(fl), F,
                                          1 if drop else 0, nt, _ptr(detect), _ptr(events), _ptr(words),
                                          _ptr(lastreg))
        if rc:
            raise ValueError(f"oracle_fault_sim_ex failed with {rc}")
        return detect, events, words, lastreg


def _load() -> OracleLib:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = OracleLib(_LIB_PATH)
    return _lib


def compile_variant(source_text: str, out_dir: str, name: str) -> OracleLib:
    """Compile modified oracle source (used to plant mistakes in tests)."""
    src = os.path.join(out_dir, name + ".c")
    with open(src, "w") as f:
        f.write(source_text)
    return OracleLib(_compile(src, os.path.join(out_dir, name + ".so")))


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


def golden(design, stimulus: np.ndarray, T: int) -> np.ndarray:
    """Golden trace G[t][n] (uint64) of the fault-free machine for cycles 0..T-1."""
    return _load().golden(design, stimulus, T)


def fault_sim(design, stimulus: np.ndarray, T: int, faults: np.ndarray, *, G: np.ndarray | None = None,
              drop: bool = True, variant: int = 1, nthreads: int | None = None):
    """Per-fault first detect cycle (0xFFFFFFFF = undetected) and event count.

    variant 0 simulates every node in every cycle; variant 1 only the nodes
    with a divergent input.  Both re-run each fault from cycle 0.
    """
    return _load().fault_sim(design, stimulus, T, faults, G=G, drop=drop, variant=variant,
                             nthreads=nthreads)


def fault_sim_stats(design, stimulus: np.ndarray, T: int, faults: np.ndarray, *, G: np.ndarray | None = None,
                    drop: bool = True, variant: int = 1, nthreads: int | None = None):
    """fault_sim plus two statistics per fault: the algorithmic memory words of
    the byte model (w(site) per simulated cycle, (k + 2) w(n) per event at a
    node with k operands, 2 w(r) more per divergent register and cycle; w = 2
    words for nodes wider than 32 bits, else 1), and the last cycle in which
    some register's state diverges (0xFFFFFFFF if none).  Returns
    (detect, events, words, lastreg)."""
    return _load().fault_sim_stats(design, stimulus, T, faults, G=G, drop=drop, variant=variant,
                                   nthreads=nthreads)


def fault_cycles(detect: np.ndarray, T: int) -> int:
    """Fault-cycles: T for an undetected fault, detect cycle + 1 otherwise."""
    d = detect.astype(np.int64)
    und = detect == UNDETECTED
    return int(np.where(und, T, d + 1).sum())
