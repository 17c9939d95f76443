"""riros_fault_sim_noalloc, the entry point for callers that cannot allocate
device memory, against riros_fault_sim in plain mode through the C ABI: two
calls in a row, the second with a smaller design and fault list, and the
rejection of what it cannot run."""
import ctypes

import numpy as np
import pytest
import torch

from helpers import Builder
from paper_2508_16376_amd import riros
from paper_2508_16376_amd import workloads as W

pytestmark = pytest.mark.gpu


def _buffers(w):
    dev = torch.device("cuda:0")
    F = w.faults.size
    return (torch.from_numpy(w.faults.view(np.uint8).copy()).to(dev), torch.empty(F, dtype=torch.int32, device=dev),
            torch.empty(F, dtype=torch.int64, device=dev), torch.empty(F, dtype=torch.int64, device=dev),
            torch.zeros(riros.COVERAGE_FIELDS, dtype=torch.int64, device=dev))


def _host(t, dt):
    return t.cpu().numpy().view(dt).copy()


def test_noalloc_equals_fault_sim_on_two_calls():
    s = torch.cuda.current_stream()
    for w in (W.medium(seed=881, F=6000, T=400, n_nodes=8000), W.tiny(F=700, T=100)):
        print(f"[noalloc] {w.name}: N={w.design.num_nodes} T={w.T} F={w.faults.size}", flush=True)
        d = riros.Design(w.design)
        g = riros.Golden(d, w.stimulus, w.T)
        f, det, ev, wk, cov = _buffers(w)
        riros.fault_sim_device(d, g, f, w.faults.size, det, ev, cov,
                               riros.make_opts(riros.MODE_PLAIN, True, True, stream=s, words=wk))
        torch.cuda.synchronize()
        ref = (_host(det, np.uint32), _host(ev, np.uint64), _host(wk, np.uint64), cov.cpu().numpy().copy())
        f2, det2, ev2, wk2, cov2 = _buffers(w)
        riros.fault_sim_noalloc(d, g, f2, w.faults.size, det2, ev2, cov2,
                                riros.make_opts(riros.MODE_PLAIN, True, True, stream=s, words=wk2))
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_host(det2, np.uint32), ref[0])
        np.testing.assert_array_equal(_host(ev2, np.uint64), ref[1])
        np.testing.assert_array_equal(_host(wk2, np.uint64), ref[2])
        np.testing.assert_array_equal(cov2.cpu().numpy(), ref[3])
        # without the optional outputs: same detect cycles, coverage without words
        det3 = torch.empty_like(det2)
        cov3 = torch.zeros_like(cov2)
        riros.fault_sim_noalloc(d, g, f2, w.faults.size, det3, None, cov3,
                                riros.make_opts(riros.MODE_PLAIN, False, True, stream=s))
        torch.cuda.synchronize()
        nd, _, _ = riros.fault_sim(d, g, w.faults, mode=riros.MODE_PLAIN, drop=False)
        np.testing.assert_array_equal(_host(det3, np.uint32), nd)
        assert int(cov3[4]) == 0 and int(cov3[1]) == w.faults.size


def test_noalloc_rejects_what_it_cannot_run():
    w = W.tiny(F=50, T=20)
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    f, det, ev, wk, cov = _buffers(w)
    for opts in (riros.make_opts(riros.MODE_TWO_D, True, True), riros.make_opts(riros.MODE_PLAIN, True, False)):
        with pytest.raises(riros.RirosError) as e:
            riros.fault_sim_noalloc(d, g, f, w.faults.size, det, ev, cov, opts)
        assert e.value.code == riros.RIROS_EINVAL
    # a design whose one-wavefront workspace (16 bytes a node) exceeds the array
    n = (128 << 20) // 16 + 1000
    b = Builder()
    x = b.pi(8)
    y = b.node(W.XOR, 8, (x, x))
    nodes = np.zeros(n, dtype=W.NODE_DTYPE)
    nodes[:2] = np.array(b.rows, dtype=W.NODE_DTYPE)
    nodes["op"][2:] = W.CONST
    nodes["width"][2:] = 1
    big = W.Design(nodes, np.array([y], dtype=np.uint32), 1, "big")
    bd = riros.Design(big)
    bg = riros.Golden(bd, np.zeros((2, 1), dtype=np.uint64), 2)
    fl = np.zeros(1, dtype=W.FAULT_DTYPE)
    fl["site"] = y
    fb = torch.from_numpy(fl.view(np.uint8).copy()).cuda()
    with pytest.raises(riros.RirosError) as e:
        riros.fault_sim_noalloc(bd, bg, fb, 1, det, ev, cov, riros.make_opts(riros.MODE_PLAIN, True, True))
    assert e.value.code == riros.RIROS_EINVAL and "scratch" in str(e.value)
