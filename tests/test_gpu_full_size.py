"""Full-size parity: every fault of the heavy-tailed (200,000 faults, 5,000
cycles), large (1,000,000 faults, 10,000 cycles) and batched-campaign (64
designs) workloads against the oracle, bit-exact: detect cycle, event count
and byte-model words of each fault, and the coverage totals; and the large
workload's no-dropping sample (20,000 faults for all 10,000 cycles).

The oracle runs on the host in the same process (tests/full_size_ref.py).
The GPU runs use the benchmark's kind of launch: two-dimensional mode with
device-resident inputs and outputs, predicted priorities with a heavy
threshold, the monitor and the unified schedule; plain mode runs the same
lists.
"""
import numpy as np
import pytest
import torch

import full_size_ref as ref
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
    wk = torch.empty(F, dtype=torch.int64, device=dev)
    cov = torch.zeros(riros.COVERAGE_FIELDS, dtype=torch.int64, device=dev)
    opts.words = wk.data_ptr()
    riros.fault_sim_device(d, g, f_dev, F, det, ev, cov, opts)
    torch.cuda.synchronize()
    return (det.cpu().numpy().view(np.uint32).copy(), ev.cpu().numpy().view(np.uint64).copy(),
            wk.cpu().numpy().view(np.uint64).copy(), cov.cpu().numpy().astype(np.int64))


def _compare(name, w, det, ev, wk, cov, odet, oev, owk):
    bad = np.flatnonzero((det != odet) | (ev != oev) | (wk != owk))
    assert bad.size == 0, (f"{name}: {bad.size} faults differ from the oracle, first {bad[:5].tolist()}: "
                           f"gpu {det[bad[:5]].tolist()} {ev[bad[:5]].tolist()} oracle {odet[bad[:5]].tolist()} "
                           f"{oev[bad[:5]].tolist()}")
    assert cov[0] == int((odet != UND).sum()) and cov[1] == w.faults.size
    assert cov[2] == ref.fault_cycles(odet, w.T)
    assert cov[3] == int(oev.sum()) and cov[4] == int(owk.sum())


def _priorities(d, g, w, seed=11):
    """Priorities as the benchmark computes them: features, then network
    inference (seeded initial weights here; any priority gives the same
    results)."""
    feats = riros.features(d, g, w.faults)
    wts = np.concatenate([W.mlp_init_weights(seed), np.zeros(6, np.float32), np.ones(6, np.float32)])
    return riros.mlp_predict(wts, feats)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["heavy_tailed", "large"])
def test_full_size_every_fault(name):
    w, odet, oev, owk = ref.single(name)
    print(f"[full-size] {name}: N={w.design.num_nodes} T={w.T} F={w.faults.size}", flush=True)
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    pred = _priorities(d, g, w)
    prio = torch.from_numpy(np.ascontiguousarray(pred, np.float32)).cuda()
    s = torch.cuda.current_stream()
    opts = riros.make_opts(riros.MODE_TWO_D, True, True, stream=s, priority=prio,
                           theta=float(np.quantile(pred, 0.99)), monitor_rate=1.0, light_cap=8, waves_per_cu=12,
                           unified=1)
    _compare(name + " two-dimensional", w, *_device_run(d, g, w, opts), odet, oev, owk)
    # The kind of schedule the benchmark's tuner picks on these lists: no
    # heavy prefix, capacity 4, lanes in lockstep, the queue's head dealt out
    # in groups of 8, workgroups of four wavefronts sharing one structural
    # workspace.
    print(f"[full-size] {name}: lockstep, dealt queue", flush=True)
    opts = riros.make_opts(riros.MODE_TWO_D, True, True, stream=s, priority=prio, light_cap=4, waves_per_cu=12,
                           unified=1, struct_share=4, lockstep=1, deal=8)
    _compare(name + " two-dimensional (lockstep, dealt)", w, *_device_run(d, g, w, opts), odet, oev, owk)
    # The schedules the tuner picks since head batches of 64 joined its
    # space: free-running lanes, head batches filling all 64 lanes, with the
    # monitor at 4 and no structural work in launch A, or the unified
    # schedule with the monitor off and workspaces shared by four.
    for kw in ({"unified": 0, "monitor_rate": 4.0, "waves_per_cu": 8, "struct_share": 2},
               {"unified": 1, "monitor_rate": 0.0, "waves_per_cu": 16, "struct_share": 4}):
        print(f"[full-size] {name}: head batches of 64, {kw}", flush=True)
        opts = riros.make_opts(riros.MODE_TWO_D, True, True, stream=s, priority=prio, light_cap=4, heavy_wg=64,
                               lockstep=0, head_lanes=64, **kw)
        _compare(name + f" two-dimensional (head batches of 64, {kw})", w, *_device_run(d, g, w, opts),
                 odet, oev, owk)
    print(f"[full-size] {name}: plain", flush=True)
    _compare(name + " plain", w, *_device_run(d, g, w, riros.make_opts(riros.MODE_PLAIN, True, True, stream=s)),
             odet, oev, owk)


@pytest.mark.timeout(600)
def test_full_size_no_drop_sample():
    """The benchmark's no-dropping leg: its 20,000-fault sample of the large
    workload, every fault simulated for all 10,000 cycles, against the
    oracle without dropping, under the drop-mode schedule and the one its
    no-dropping tuning picks (capacity 8, the monitor off, unified)."""
    w, odet, oev, owk = ref.no_drop_sample("large", 20000)
    print(f"[full-size] large without dropping: F={w.faults.size}", flush=True)
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    pred = _priorities(d, g, w)
    prio = torch.from_numpy(np.ascontiguousarray(pred, np.float32)).cuda()
    s = torch.cuda.current_stream()
    base = {"heavy_wg": 64, "lockstep": 0, "head_lanes": 64, "waves_per_cu": 12}
    for kw in ({"light_cap": 4, "unified": 0, "monitor_rate": 4.0, "struct_share": 2},
               {"light_cap": 8, "unified": 1, "monitor_rate": 0.0, "struct_share": 4}):
        print(f"[full-size] large without dropping: {kw}", flush=True)
        opts = riros.make_opts(riros.MODE_TWO_D, False, True, stream=s, priority=prio, **base, **kw)
        _compare(f"large without dropping ({kw})", w, *_device_run(d, g, w, opts), odet, oev, owk)


@pytest.mark.timeout(600)
def test_full_size_campaign_every_fault():
    """The 64-design campaign in one graph launch (predicted priorities with a
    heavy threshold, monitor, unified schedule), two replays; every fault of
    every design against the oracle."""
    refs = ref.campaign()
    print(f"[full-size] campaign: {sum(r[0].faults.size for r in refs)} faults", flush=True)
    ws = [r[0] for r in refs]
    ds = [riros.Design(w.design) for w in ws]
    gs = [riros.Golden(d, w.stimulus, w.T) for d, w in zip(ds, ws)]
    prios = [_priorities(d, g, w) for d, g, w in zip(ds, gs, ws)]
    theta = float(np.quantile(np.concatenate(prios), 0.95))
    b = riros.Batch(ds, gs, [w.faults for w in ws], prios, theta=theta, monitor_rate=2.0, unified=1)
    for rep in range(2):
        b.launch()
        for i, (w, odet, oev, owk) in enumerate(refs):
            wk = np.empty(w.faults.size, dtype=np.uint64)
            det, ev, cov = b.read(i, words_out=wk)
            c = np.array([cov["detected"], cov["total"], cov["fault_cycles"], cov["events"], cov["words"]])
            _compare(f"campaign design {i} replay {rep}", w, det, ev, wk, c, odet, oev, owk)
    b.close()
