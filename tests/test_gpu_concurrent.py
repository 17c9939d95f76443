"""GPU parity of the concurrent (node-major) mode beyond the shared matrix of
tests/test_gpu_parity.py: wavefronts that take several groups in turn (their
stamps carry over), a workspace that grows and is reused, device-resident
inputs and outputs, and the heavy-tailed and large lists at full size
against the oracle's stored samples."""
import numpy as np
import pytest
import torch

import oracle
import full_size_ref as ref
from paper_2508_16376_amd import riros
from paper_2508_16376_amd import workloads as W

pytestmark = pytest.mark.gpu
UND = riros.UNDETECTED
CONC = riros.MODE_CONCURRENT


@pytest.fixture(scope="module")
def many():
    # 40,000 faults = 625 groups of 64: more groups than a compute unit's
    # share of wavefronts at one or two per compute unit
    return W.medium(seed=778, F=40000, T=300, n_nodes=3000)


@pytest.fixture(scope="module")
def many_oracle(many):
    w = many
    return {drop: oracle.fault_sim(w.design, w.stimulus, w.T, w.faults, drop=drop) for drop in (True, False)}


def test_groups_share_wavefronts_and_workspace_grows(many, many_oracle):
    """One, then all, then two wavefronts per compute unit on one design
    handle: each wavefront takes many groups with one stamp counter, the
    workspace is reallocated for more wavefronts and reused for fewer."""
    w = many
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    for wpc in (1, 0, 2):
        for drop in (True, False):
            print(f"[concurrent] waves_per_cu={wpc} drop={drop}", flush=True)
            det, ev, cov = riros.fault_sim(d, g, w.faults, mode=CONC, drop=drop, waves_per_cu=wpc)
            odet, oev = many_oracle[drop]
            np.testing.assert_array_equal(det, odet)
            np.testing.assert_array_equal(ev, oev)
            assert cov["events"] == int(oev.sum())


def test_other_modes_then_concurrent_on_one_handle(many, many_oracle):
    w = many
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    odet, oev = many_oracle[True]
    for mode in (riros.MODE_TWO_D, CONC, riros.MODE_PLAIN, CONC):
        det, ev, _ = riros.fault_sim(d, g, w.faults[:5000], mode=mode)
        np.testing.assert_array_equal(det, odet[:5000])
        np.testing.assert_array_equal(ev, oev[:5000])


def test_device_io(many, many_oracle):
    w = many
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    dev = torch.device("cuda:0")
    F = w.faults.size
    f_dev = torch.from_numpy(w.faults.view(np.uint8).copy()).to(dev)
    det = torch.empty(F, dtype=torch.int32, device=dev)
    ev = torch.empty(F, dtype=torch.int64, device=dev)
    cov = torch.zeros(riros.COVERAGE_FIELDS, dtype=torch.int64, device=dev)
    opts = riros.make_opts(CONC, True, True, stream=torch.cuda.current_stream())
    riros.fault_sim_device(d, g, f_dev, F, det, ev, cov, opts)
    torch.cuda.synchronize()
    odet, oev = many_oracle[True]
    np.testing.assert_array_equal(det.cpu().numpy().view(np.uint32), odet)
    np.testing.assert_array_equal(ev.cpu().numpy().view(np.uint64), oev)
    c = cov.cpu().numpy()
    assert c[0] == int((odet != UND).sum()) and c[1] == F and c[3] == int(oev.sum())


def test_one_site_many_faults():
    """Every fault of the list on one node (one group shares a single
    frontier), with flips in every cycle of a window."""
    w = W.medium(seed=779, F=10, T=200, n_nodes=2000)
    site = int(w.faults["site"][3])
    width = int(w.design.nodes["width"][site])
    rows = []
    for b in range(width):
        for stuck in (0, 1):
            rows.append((site, b, stuck, 0))
        for t0 in (0, 5, 64, 199):
            rows.append((site, b, 2, t0))
    fl = np.zeros(len(rows), dtype=w.faults.dtype)
    for i, (s_, b, st, t0) in enumerate(rows):
        fl[i]["site"], fl[i]["bit"], fl[i]["stuck"], fl[i]["t0"] = s_, b, st, t0
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    for drop in (True, False):
        det, ev, _ = riros.fault_sim(d, g, fl, mode=CONC, drop=drop)
        odet, oev = oracle.fault_sim(w.design, w.stimulus, w.T, fl, drop=drop)
        np.testing.assert_array_equal(det, odet)
        np.testing.assert_array_equal(ev, oev)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["heavy_tailed", "large"])
def test_full_size_every_fault(name):
    """Every fault of the full-size lists against the oracle, and the same
    results as the two-dimensional schedule."""
    w, odet, oev, owk = ref.single(name)
    print(f"[concurrent full-size] {name}: N={w.design.num_nodes} T={w.T} F={w.faults.size}", flush=True)
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    wk = np.empty(w.faults.size, dtype=np.uint64)
    det, ev, cov = riros.fault_sim(d, g, w.faults, mode=CONC, words_out=wk)
    np.testing.assert_array_equal(det, odet)
    np.testing.assert_array_equal(ev, oev)
    np.testing.assert_array_equal(wk, owk)
    assert cov["words"] == int(owk.sum()) and cov["events"] == int(oev.sum())
    print(f"[concurrent full-size] {name}: two-dimensional", flush=True)
    tdet, tev, tcov = riros.fault_sim(d, g, w.faults, mode=riros.MODE_TWO_D, monitor_rate=2.0, unified=1)
    np.testing.assert_array_equal(det, tdet)
    np.testing.assert_array_equal(ev, tev)
    assert cov == tcov
