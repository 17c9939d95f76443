"""Python binding of the C interface in include/riros.h (argument marshalling only).

Every simulation step runs in the HIP library ``_build/libriros.so``; this
module only converts arguments.  Importing it raises if the library has not
been built (``python -m paper_2508_16376_amd.build``); there is no fallback.
Device buffers and streams may be passed as torch tensors / streams, whose
pointers are handed to the library unchanged.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libriros.so")

RIROS_OK = 0
RIROS_EINVAL = -1
RIROS_ECYCLE = -2
RIROS_ENOMEM = -3
RIROS_EDEVICE = -4
UNDETECTED = 0xFFFFFFFF
MODE_PLAIN = 0
MODE_TWO_D = 1
MODE_CONCURRENT = 2

EXPORTED = ["riros_load_design", "riros_free_design", "riros_golden_sim", "riros_free_golden",
            "riros_golden_read", "riros_fault_sim", "riros_design_info", "riros_last_kernel_ms",
            "riros_last_error", "riros_features", "riros_mlp_train", "riros_mlp_predict", "riros_mlp_grad",
            "riros_batch_create", "riros_batch_launch", "riros_batch_read", "riros_batch_free",
            "riros_peak_hbm", "riros_peak_valu", "riros_golden_sim_many", "riros_fault_sim_noalloc"]
N_FEATURES = 6
MLP_PARAMS = 4673
MLP_WEIGHTS = MLP_PARAMS + 12


class RirosError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"riros error {code}: {msg}")
        self.code = code


class _DesignDesc(ctypes.Structure):
    _fields_ = [("num_nodes", ctypes.c_uint32), ("nodes", ctypes.c_void_p),
                ("num_pi", ctypes.c_uint32), ("num_po", ctypes.c_uint32), ("po", ctypes.c_void_p)]


class SimOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("drop", ctypes.c_int32), ("io_on_device", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("priority", ctypes.c_void_p), ("theta", ctypes.c_float),
                ("light_cap", ctypes.c_int32), ("unified", ctypes.c_int32), ("monitor_rate", ctypes.c_float),
                ("struct_share", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("words", ctypes.c_void_p), ("campaign_golden", ctypes.c_int32),
                ("heavy_wg", ctypes.c_int32), ("lockstep", ctypes.c_int32), ("deal", ctypes.c_int32),
                ("head_lanes", ctypes.c_int32), ("xcd_queues", ctypes.c_int32)]


class TrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class Coverage(ctypes.Structure):
    _fields_ = [("detected", ctypes.c_uint64), ("total", ctypes.c_uint64),
                ("fault_cycles", ctypes.c_uint64), ("events", ctypes.c_uint64), ("words", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def _hip_runtimes_mapped() -> set[str]:
    try:
        with open("/proc/self/maps") as f:
            return {line.split()[-1] for line in f if "libamdhip64" in line}
    except OSError:
        return set()


def lib():
    """The loaded library; raises when it is missing (no CPU fallback exists).

    torch is imported first so that its HIP runtime is the one the library
    binds to (both carry the soname libamdhip64.so.7); the library's kernels
    then share streams and device memory with torch tensors.
    """
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run python -m paper_2508_16376_amd.build)")
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        runtimes = _hip_runtimes_mapped()
        if len(runtimes) > 1:
            raise RuntimeError(f"two HIP runtimes are loaded in this process: {sorted(runtimes)}")
        P, U, I = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
        L.riros_load_design.argtypes = [ctypes.POINTER(_DesignDesc), ctypes.POINTER(P)]
        L.riros_load_design.restype = I
        L.riros_free_design.argtypes = [P]
        L.riros_free_design.restype = None
        L.riros_golden_sim.argtypes = [P, P, U, P, ctypes.POINTER(P)]
        L.riros_golden_sim.restype = I
        L.riros_golden_sim_many.argtypes = [U, P, P, P, P, P]
        L.riros_golden_sim_many.restype = I
        L.riros_free_golden.argtypes = [P]
        L.riros_free_golden.restype = None
        L.riros_golden_read.argtypes = [P, U, U, P]
        L.riros_golden_read.restype = I
        L.riros_fault_sim.argtypes = [P, P, P, U, ctypes.POINTER(SimOpts), P, P, ctypes.POINTER(Coverage)]
        L.riros_fault_sim.restype = I
        L.riros_fault_sim_noalloc.argtypes = [P, P, P, U, ctypes.POINTER(SimOpts), P, P, ctypes.POINTER(Coverage)]
        L.riros_fault_sim_noalloc.restype = I
        L.riros_design_info.argtypes = [P, ctypes.POINTER(U), ctypes.POINTER(U), ctypes.POINTER(U)]
        L.riros_design_info.restype = I
        L.riros_last_kernel_ms.argtypes = [ctypes.POINTER(ctypes.c_float)]
        L.riros_last_kernel_ms.restype = I
        L.riros_last_error.argtypes = []
        L.riros_last_error.restype = ctypes.c_char_p
        L.riros_features.argtypes = [P, P, P, U, P, ctypes.c_int32, P]
        L.riros_features.restype = I
        L.riros_mlp_train.argtypes = [P, P, U, ctypes.POINTER(TrainCfg), P, P, P]
        L.riros_mlp_train.restype = I
        L.riros_mlp_predict.argtypes = [P, P, U, P, ctypes.c_int32, P]
        L.riros_mlp_predict.restype = I
        L.riros_mlp_grad.argtypes = [P, P, P, U, P, P, P]
        L.riros_mlp_grad.restype = I
        L.riros_batch_create.argtypes = [U, P, P, P, P, P, ctypes.POINTER(SimOpts), ctypes.POINTER(P)]
        L.riros_batch_create.restype = I
        L.riros_batch_launch.argtypes = [P, P]
        L.riros_batch_launch.restype = I
        L.riros_batch_read.argtypes = [P, U, P, P, P, ctypes.POINTER(Coverage)]
        L.riros_batch_read.restype = I
        L.riros_batch_free.argtypes = [P]
        L.riros_batch_free.restype = None
        L.riros_peak_hbm.argtypes = [ctypes.c_uint64, I, ctypes.POINTER(ctypes.c_double), P]
        L.riros_peak_hbm.restype = I
        L.riros_peak_valu.argtypes = [I, ctypes.POINTER(ctypes.c_double), P]
        L.riros_peak_valu.restype = I
        _lib = L
    return _lib


def _check(rc: int):
    if rc != RIROS_OK:
        raise RirosError(rc, lib().riros_last_error().decode(errors="replace"))


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_ptr(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


class Design:
    """riros_load_design handle."""

    def __init__(self, design):
        self._nodes = np.ascontiguousarray(design.nodes)
        self._po = np.ascontiguousarray(design.po, dtype=np.uint32)
        desc = _DesignDesc(self._nodes.size, _ptr(self._nodes), design.num_pi, self._po.size, _ptr(self._po))
        h = ctypes.c_void_p()
        _check(lib().riros_load_design(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.num_pi = design.num_pi

    def info(self):
        n, l, r = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
        _check(lib().riros_design_info(self.handle, ctypes.byref(n), ctypes.byref(l), ctypes.byref(r)))
        return {"nodes": n.value, "levels": l.value, "regs": r.value}

    def close(self):
        if self.handle:
            lib().riros_free_design(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Golden:
    """riros_golden_sim handle (trace resident on the device)."""

    def __init__(self, design: Design, stimulus: np.ndarray, T: int, stream=None, _handle=None):
        self.design = design
        self.T = T
        if _handle is not None:
            self.handle = _handle
            return
        stim = np.ascontiguousarray(stimulus[:T], dtype=np.uint64)
        if stim.shape[0] < T:
            raise ValueError("stimulus has fewer rows than T")
        h = ctypes.c_void_p()
        _check(lib().riros_golden_sim(design.handle, _ptr(stim), T, _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    @staticmethod
    def many(designs, stimuli, Ts, stream=None):
        """riros_golden_sim_many: the golden traces of many designs in one launch."""
        n = len(designs)
        stims = [np.ascontiguousarray(s[:T], dtype=np.uint64) for s, T in zip(stimuli, Ts)]
        for s_, T in zip(stims, Ts):
            if s_.shape[0] < T:
                raise ValueError("stimulus has fewer rows than T")
        dh = (ctypes.c_void_p * n)(*[d.handle.value for d in designs])
        sp = (ctypes.c_void_p * n)(*[s_.ctypes.data for s_ in stims])
        Ta = np.ascontiguousarray(Ts, dtype=np.uint32)
        out = (ctypes.c_void_p * n)()
        _check(lib().riros_golden_sim_many(n, dh, sp, _ptr(Ta), _stream_ptr(stream), out))
        return [Golden(d, None, int(T), _handle=ctypes.c_void_p(out[i])) for i, (d, T) in enumerate(zip(designs, Ts))]

    def read(self, t0: int = 0, nt: int | None = None) -> np.ndarray:
        nt = self.T - t0 if nt is None else nt
        N = self.design.info()["nodes"]
        out = np.empty((nt, N), dtype=np.uint64)
        _check(lib().riros_golden_read(self.handle, t0, nt, _ptr(out)))
        return out

    def close(self):
        if self.handle:
            lib().riros_free_golden(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Words of device memory per riros_coverage (detected, total, fault_cycles, events, words).
COVERAGE_FIELDS = 5


def make_opts(mode=MODE_PLAIN, drop=True, io_on_device=False, waves_per_cu=0, priority=None,
              theta=math.inf, light_cap=0, unified=0, monitor_rate=0.0, stream=None, struct_share=0,
              words=None, campaign_golden=False, heavy_wg=0, lockstep=0, deal=0, head_lanes=0,
              xcd_queues=0) -> SimOpts:
    return SimOpts(mode, 1 if drop else 0, 1 if io_on_device else 0, waves_per_cu, _ptr(priority),
                   theta, light_cap, unified, monitor_rate, struct_share, _stream_ptr(stream), _ptr(words),
                   1 if campaign_golden else 0, heavy_wg, int(lockstep), deal, head_lanes, int(xcd_queues))


def fault_sim(design: Design, golden: Golden, faults: np.ndarray, *, mode=MODE_PLAIN, drop=True,
              waves_per_cu=0, priority=None, theta=math.inf, light_cap=0, unified=0, monitor_rate=0.0,
              stream=None, with_events=True, struct_share=0, words_out=None, heavy_wg=0, lockstep=0, deal=0,
              head_lanes=0, xcd_queues=0):
    """riros_fault_sim on host arrays: returns (detect, events, coverage dict).
    words_out (optional uint64[F]) receives the per-fault byte-model words."""
    fl = np.ascontiguousarray(faults)
    F = fl.size
    detect = np.empty(F, dtype=np.uint32)
    events = np.empty(F, dtype=np.uint64) if with_events else None
    pr = None if priority is None else np.ascontiguousarray(priority, dtype=np.float32)
    if words_out is not None:
        assert words_out.dtype == np.uint64 and words_out.size == F and words_out.flags.c_contiguous
    opts = make_opts(mode, drop, False, waves_per_cu, pr, theta, light_cap, unified, monitor_rate, stream,
                     struct_share, words_out, heavy_wg=heavy_wg, lockstep=lockstep, deal=deal,
                     head_lanes=head_lanes, xcd_queues=xcd_queues)
    cov = Coverage()
    _check(lib().riros_fault_sim(design.handle, golden.handle, _ptr(fl), F, ctypes.byref(opts), _ptr(detect),
                                 _ptr(events), ctypes.byref(cov)))
    return detect, events, cov.as_dict()


def fault_sim_device(design: Design, golden: Golden, faults_dev, F: int, detect_dev, events_dev, cov_dev,
                     opts: SimOpts):
    """riros_fault_sim with device-resident buffers (asynchronous on opts.stream)."""
    opts.io_on_device = 1
    _check(lib().riros_fault_sim(design.handle, golden.handle, _ptr(faults_dev), F, ctypes.byref(opts),
                                 _ptr(detect_dev), _ptr(events_dev),
                                 ctypes.cast(_ptr(cov_dev), ctypes.POINTER(Coverage)) if cov_dev is not None
                                 else None))


def fault_sim_noalloc(design: Design, golden: Golden, faults_dev, F: int, detect_dev, events_dev, cov_dev,
                      opts: SimOpts):
    """riros_fault_sim_noalloc: plain mode, device-resident buffers, no device
    allocation (asynchronous on opts.stream after the fault check)."""
    _check(lib().riros_fault_sim_noalloc(design.handle, golden.handle, _ptr(faults_dev), F, ctypes.byref(opts),
                                         _ptr(detect_dev), _ptr(events_dev),
                                         ctypes.cast(_ptr(cov_dev), ctypes.POINTER(Coverage))
                                         if cov_dev is not None else None))


def last_kernel_ms() -> float:
    ms = ctypes.c_float()
    _check(lib().riros_last_kernel_ms(ctypes.byref(ms)))
    return float(ms.value)


def features(design: Design, golden: Golden, faults: np.ndarray) -> np.ndarray:
    """riros_features on host arrays: float32[F][6]."""
    fl = np.ascontiguousarray(faults)
    out = np.empty((fl.size, N_FEATURES), dtype=np.float32)
    _check(lib().riros_features(design.handle, golden.handle, _ptr(fl), fl.size, _ptr(out), 0, None))
    return out


def features_device(design: Design, golden: Golden, faults_dev, F: int, out_dev, stream=None):
    _check(lib().riros_features(design.handle, golden.handle, _ptr(faults_dev), F, _ptr(out_dev), 1,
                                _stream_ptr(stream)))


def mlp_train(feats: np.ndarray, y: np.ndarray, init_params: np.ndarray, *, epochs=10, batch=4096, lr=1e-3,
              beta1=0.9, beta2=0.999, eps=1e-8):
    """riros_mlp_train: returns (weights float32[MLP_WEIGHTS], per-step losses)."""
    x = np.ascontiguousarray(feats, dtype=np.float32)
    yy = np.ascontiguousarray(y, dtype=np.float32)
    S = x.shape[0]
    w = np.zeros(MLP_WEIGHTS, dtype=np.float32)
    w[:MLP_PARAMS] = init_params[:MLP_PARAMS]
    B = min(batch, S)
    steps = epochs * ((S + B - 1) // B)
    losses = np.empty(steps, dtype=np.float32)
    cfg = TrainCfg(epochs, batch, lr, beta1, beta2, eps)
    _check(lib().riros_mlp_train(_ptr(x), _ptr(yy), S, ctypes.byref(cfg), _ptr(w), _ptr(losses), None))
    return w, losses


def mlp_predict(weights: np.ndarray, feats: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(weights, dtype=np.float32)
    x = np.ascontiguousarray(feats, dtype=np.float32)
    out = np.empty(x.shape[0], dtype=np.float32)
    _check(lib().riros_mlp_predict(_ptr(w), _ptr(x), x.shape[0], _ptr(out), 0, None))
    return out


def mlp_predict_device(weights_dev, feats_dev, F: int, out_dev, stream=None):
    _check(lib().riros_mlp_predict(_ptr(weights_dev), _ptr(feats_dev), F, _ptr(out_dev), 1, _stream_ptr(stream)))


def mlp_grad(weights: np.ndarray, feats: np.ndarray, y: np.ndarray):
    w = np.ascontiguousarray(weights, dtype=np.float32)
    x = np.ascontiguousarray(feats, dtype=np.float32)
    yy = np.ascontiguousarray(y, dtype=np.float32)
    g = np.empty(MLP_PARAMS, dtype=np.float32)
    loss = np.empty(1, dtype=np.float32)
    _check(lib().riros_mlp_grad(_ptr(w), _ptr(x), _ptr(yy), x.shape[0], _ptr(g), _ptr(loss), None))
    return g, float(loss[0])


class Batch:
    """riros_batch_create handle: a campaign of designs run as one graph launch."""

    def __init__(self, designs, goldens, fault_lists, priorities=None, *, drop=True, waves_per_cu=0,
                 theta=math.inf, light_cap=0, monitor_rate=0.0, unified=0, struct_share=0, campaign_golden=False,
                 heavy_wg=0, lockstep=0, deal=0, head_lanes=0, xcd_queues=0):
        n = len(designs)
        fls = [np.ascontiguousarray(f) for f in fault_lists]
        self.F = [int(f.size) for f in fls]
        dh = (ctypes.c_void_p * n)(*[d.handle.value for d in designs])
        gh = (ctypes.c_void_p * n)(*[g.handle.value for g in goldens])
        fp = (ctypes.c_void_p * n)(*[f.ctypes.data for f in fls])
        Fa = np.asarray(self.F, dtype=np.uint32)
        pp = None
        keep = []
        if priorities is not None:
            prs = [None if p is None else np.ascontiguousarray(p, dtype=np.float32) for p in priorities]
            keep = prs
            pp = (ctypes.c_void_p * n)(*[0 if p is None else p.ctypes.data for p in prs])
        opts = make_opts(MODE_TWO_D, drop, False, waves_per_cu, None, theta, light_cap, unified, monitor_rate, None,
                         struct_share, campaign_golden=campaign_golden, heavy_wg=heavy_wg, lockstep=lockstep,
                         deal=deal, head_lanes=head_lanes, xcd_queues=xcd_queues)
        h = ctypes.c_void_p()
        _check(lib().riros_batch_create(n, dh, gh, fp, _ptr(Fa), pp, ctypes.byref(opts), ctypes.byref(h)))
        del keep
        self.handle = h
        self.n = n
        self.designs, self.goldens = designs, goldens   # keep the handles alive

    def launch(self, stream=None):
        _check(lib().riros_batch_launch(self.handle, _stream_ptr(stream)))

    def read(self, i, words_out=None):
        """(detect, events, coverage dict) of design i; words_out (optional
        uint64[F[i]]) receives its per-fault byte-model words."""
        det = np.empty(self.F[i], dtype=np.uint32)
        ev = np.empty(self.F[i], dtype=np.uint64)
        if words_out is not None:
            assert words_out.dtype == np.uint64 and words_out.size == self.F[i]
        cov = Coverage()
        _check(lib().riros_batch_read(self.handle, i, _ptr(det), _ptr(ev), _ptr(words_out), ctypes.byref(cov)))
        return det, ev, cov.as_dict()

    def close(self):
        if self.handle:
            lib().riros_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def peak_hbm_gbs(nbytes: int = 2 << 30, reps: int = 5, stream=None) -> float:
    """riros_peak_hbm: best streaming-copy rate in GB/s (bytes read + written)."""
    out = ctypes.c_double()
    rc = lib().riros_peak_hbm(nbytes, reps, ctypes.byref(out), _stream_ptr(stream))
    if rc:
        raise RirosError(rc, "HBM probe failed")
    return float(out.value)


def peak_valu_ops(reps: int = 5, stream=None) -> float:
    """riros_peak_valu: best int32 vector-ALU rate, instructions per second per lane."""
    out = ctypes.c_double()
    rc = lib().riros_peak_valu(reps, ctypes.byref(out), _stream_ptr(stream))
    if rc:
        raise RirosError(rc, "VALU probe failed")
    return float(out.value)
