"""Full-size parity for the heavy-tailed and large workloads.

The oracle cannot finish these fault lists inside a test, so its results on a
seeded sample of each list were stored by tests/golden/make_expected.py (which
calls only the oracle).  Here the whole list runs on the GPU, in the launch
configuration the benchmark times (two-dimensional mode, device-resident
inputs and outputs, predicted priorities with a heavy threshold, the
monitor on) and in plain mode; the sampled faults must match the oracle
exactly and the two modes must agree on every fault.
"""
import numpy as np
import pytest
import torch

from golden import make_expected
from paper_2508_16376_amd import riros
from paper_2508_16376_amd import workloads as W

pytestmark = pytest.mark.gpu
UND = riros.UNDETECTED


def _device_run(d, g, w, opts):
    dev = torch.device("cuda:0")
    F = w.faults.size
    f_dev = torch.from_numpy(w.faults.view(np.uint8).copy()).to(dev)
    det = torch.empty(F, dtype=torch.int32, device=dev)
    ev = torch.empty(F, dtype=torch.int64, device=dev)
    cov = torch.zeros(4, dtype=torch.int64, device=dev)
    riros.fault_sim_device(d, g, f_dev, F, det, ev, cov, opts)
    torch.cuda.synchronize()
    return (det.cpu().numpy().view(np.uint32).copy(), ev.cpu().numpy().view(np.uint64).copy(),
            cov.cpu().numpy().astype(np.int64))


@pytest.mark.parametrize("name", ["heavy_tailed", "large"])
def test_full_size_against_stored_oracle_sample(name):
    digest, idx, odet, oev = make_expected.read(name)
    w = make_expected.MAKERS[name][0]()
    print(f"[full-size] {name}: N={w.design.num_nodes} T={w.T} F={w.faults.size} sample={idx.size}", flush=True)
    assert make_expected.workload_digest(w) == digest, \
        "the workload generator changed; rerun tests/golden/make_expected.py"
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)

    # Priorities as the benchmark computes them: features, then MLP inference
    # (seeded initial weights here; any priority must give the same results).
    feats = riros.features(d, g, w.faults)
    wts = np.concatenate([W.mlp_init_weights(11), np.zeros(6, np.float32), np.ones(6, np.float32)])
    pred = riros.mlp_predict(wts, feats)
    prio = torch.from_numpy(np.ascontiguousarray(pred, np.float32)).cuda()
    theta = float(np.quantile(pred, 0.99))
    s = torch.cuda.current_stream()
    opts = riros.make_opts(riros.MODE_TWO_D, True, True, stream=s, priority=prio, theta=theta,
                           monitor_rate=1.0, light_cap=8, waves_per_cu=12, unified=1)
    det, ev, cov = _device_run(d, g, w, opts)
    np.testing.assert_array_equal(det[idx], odet)
    np.testing.assert_array_equal(ev[idx], oev)
    fc = int(np.where(det == UND, w.T, det.astype(np.int64) + 1).sum())
    assert cov[0] == int((det != UND).sum()) and cov[1] == w.faults.size
    assert cov[2] == fc and cov[3] == int(ev.sum())

    print(f"[full-size] {name}: plain", flush=True)
    pdet, pev, pcov = _device_run(d, g, w, riros.make_opts(riros.MODE_PLAIN, True, True, stream=s))
    np.testing.assert_array_equal(pdet, det)
    np.testing.assert_array_equal(pev, ev)
    np.testing.assert_array_equal(pcov, cov)
