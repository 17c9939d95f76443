"""Batched campaigns: one captured graph over many designs' faults gives, per
design, exactly the oracle's detect cycles and events, on every replay."""
import numpy as np
import pytest

import oracle
from paper_2508_16376_amd import riros
from paper_2508_16376_amd import workloads as W

pytestmark = pytest.mark.gpu


def _load(ws):
    ds = [riros.Design(w.design) for w in ws]
    gs = [riros.Golden(d, w.stimulus, w.T) for d, w in zip(ds, ws)]
    return ds, gs


@pytest.fixture(scope="module")
def small_campaign():
    ws = W.campaign(seed=424242, n=8, nodes=(300, 4000), faults=(200, 3000), cycles=(50, 400))
    refs = [oracle.fault_sim(w.design, w.stimulus, w.T, w.faults) for w in ws]
    return ws, refs


@pytest.mark.parametrize("kw", [{}, {"monitor_rate": 2.0}, {"light_cap": 4, "waves_per_cu": 3},
                                {"monitor_rate": 1.0, "unified": 1}])
def test_small_campaign_matches_oracle_on_every_replay(small_campaign, kw):
    import torch
    ws, refs = small_campaign
    ds, gs = _load(ws)
    b = riros.Batch(ds, gs, [w.faults for w in ws], **kw)
    for rep in range(3):
        b.launch()
        torch.cuda.synchronize()
        x = torch.ones(1 << 20, device="cuda").sum().item()   # unrelated work between replays
        assert x == float(1 << 20)
        for i, w in enumerate(ws):
            det, ev, cov = b.read(i)
            np.testing.assert_array_equal(det, refs[i][0], err_msg=f"replay {rep} design {i}")
            np.testing.assert_array_equal(ev, refs[i][1], err_msg=f"replay {rep} design {i}")
            assert cov["total"] == w.faults.size
            assert cov["detected"] == int((refs[i][0] != riros.UNDETECTED).sum())
            assert cov["fault_cycles"] == oracle.fault_cycles(refs[i][0], w.T)
            assert cov["events"] == int(refs[i][1].sum())


def test_small_campaign_priorities_and_heavy_split(small_campaign):
    ws, refs = small_campaign
    ds, gs = _load(ws)
    prios = [np.log2(1 + r[1].astype(np.float32)) for r in refs]
    theta = float(np.quantile(np.concatenate(prios), 0.9))
    for unified, share in ((0, 0), (1, 0), (1, 2), (1, 4)):
        b = riros.Batch(ds, gs, [w.faults for w in ws], prios, theta=theta, monitor_rate=4.0, unified=unified,
                        struct_share=share)
        for _ in range(2):
            b.launch()
            for i in range(len(ws)):
                det, ev, _ = b.read(i)
                np.testing.assert_array_equal(det, refs[i][0])
                np.testing.assert_array_equal(ev, refs[i][1])
        b.close()


def test_campaign_equals_single_design_runs(small_campaign):
    ws, refs = small_campaign
    ds, gs = _load(ws)
    b = riros.Batch(ds, gs, [w.faults for w in ws])
    b.launch()
    for i, w in enumerate(ws):
        det, ev, _ = b.read(i)
        sdet, sev, _ = riros.fault_sim(ds[i], gs[i], w.faults, mode=riros.MODE_TWO_D)
        np.testing.assert_array_equal(det, sdet)
        np.testing.assert_array_equal(ev, sev)


def test_campaign_with_flips():
    """Stuck-at faults and bit flips mixed in one campaign, on two replays."""
    ws = W.campaign(seed=515151, n=5, nodes=(300, 3000), faults=(200, 2000), cycles=(50, 300))
    fls = [np.concatenate([w.faults, W.gen_flip_faults(600 + i, w.design, 500, w.T)]) for i, w in enumerate(ws)]
    refs = [oracle.fault_sim(w.design, w.stimulus, w.T, fl) for w, fl in zip(ws, fls)]
    ds, gs = _load(ws)
    b = riros.Batch(ds, gs, fls, monitor_rate=1.0, unified=1)
    for _ in range(2):
        b.launch()
        for i in range(len(ws)):
            det, ev, _ = b.read(i)
            np.testing.assert_array_equal(det, refs[i][0])
            np.testing.assert_array_equal(ev, refs[i][1])


def test_golden_many_equals_oracle(small_campaign):
    """riros_golden_sim_many (one workgroup per design, one launch) gives each
    design the oracle's golden trace."""
    ws, _ = small_campaign
    ds = [riros.Design(w.design) for w in ws]
    gs = riros.Golden.many(ds, [w.stimulus for w in ws], [w.T for w in ws])
    for w, g in zip(ws, gs):
        np.testing.assert_array_equal(g.read(), oracle.golden(w.design, w.stimulus, w.T), err_msg=w.name)


def test_campaign_golden_in_graph_on_every_replay(small_campaign):
    """The campaign graph recomputes every golden trace before the fault
    simulation (goldens from riros_golden_sim_many); three replays with
    unrelated work between them all give the oracle's results."""
    import torch
    ws, refs = small_campaign
    ds = [riros.Design(w.design) for w in ws]
    gs = riros.Golden.many(ds, [w.stimulus for w in ws], [w.T for w in ws])
    prios = [np.log2(1 + r[1].astype(np.float32)) for r in refs]
    b = riros.Batch(ds, gs, [w.faults for w in ws], prios, theta=float(np.quantile(np.concatenate(prios), 0.9)),
                    monitor_rate=2.0, unified=1, campaign_golden=True)
    for rep in range(3):
        b.launch()
        torch.cuda.synchronize()
        assert torch.ones(1 << 20, device="cuda").sum().item() == float(1 << 20)
        for i, w in enumerate(ws):
            det, ev, _ = b.read(i)
            np.testing.assert_array_equal(det, refs[i][0], err_msg=f"replay {rep} design {i}")
            np.testing.assert_array_equal(ev, refs[i][1], err_msg=f"replay {rep} design {i}")
        np.testing.assert_array_equal(gs[0].read(), oracle.golden(ws[0].design, ws[0].stimulus, ws[0].T))
    b.close()


def test_golden_many_and_in_graph_mixing_parts_and_whole_designs():
    """A campaign whose designs take both golden paths: template designs (by
    parts) and a layered design too large for one part (one workgroup for the
    whole design).  riros_golden_sim_many and the golden recomputed inside the
    campaign graph both give the oracle's traces and results."""
    import torch
    ws = []
    for k in range(3):
        s = 737373 + 1000 * k
        d = W.gen_templates(s, n_nodes=1200 + 900 * k, name=f"tmpl{k}")
        T = 150 + 50 * k
        ws.append(W.Workload(d.name, d, W.gen_stimulus(s, d, T), W.gen_faults(s, d, 800), T))
    ws.append(W.medium(seed=838383, F=600, T=100, n_nodes=5200))
    refs = [oracle.fault_sim(w.design, w.stimulus, w.T, w.faults) for w in ws]
    ds = [riros.Design(w.design) for w in ws]
    gs = riros.Golden.many(ds, [w.stimulus for w in ws], [w.T for w in ws])
    for w, g in zip(ws, gs):
        np.testing.assert_array_equal(g.read(), oracle.golden(w.design, w.stimulus, w.T), err_msg=w.name)
    b = riros.Batch(ds, gs, [w.faults for w in ws], None, unified=1, campaign_golden=True)
    for rep in range(2):
        b.launch()
        torch.cuda.synchronize()
        for i, w in enumerate(ws):
            det, ev, _ = b.read(i)
            np.testing.assert_array_equal(det, refs[i][0], err_msg=f"replay {rep} design {i}")
            np.testing.assert_array_equal(ev, refs[i][1], err_msg=f"replay {rep} design {i}")
        for w, g in zip(ws, gs):
            np.testing.assert_array_equal(g.read(), oracle.golden(w.design, w.stimulus, w.T), err_msg=w.name)
    b.close()


def test_campaign_of_narrow_template_designs():
    """A campaign whose designs are all at most 32 bits wide (template designs:
    light lanes keep 32-bit values) with priorities, a heavy prefix on
    two-wavefront workgroups, the unified schedule, per-XCD light queues and
    lanes in lockstep, on two replays."""
    ws = []
    for k in range(4):
        s = 626262 + 1000 * k
        d = W.gen_templates(s, n_nodes=1500 + 700 * k, name=f"tmpl{k}")
        T = 300 + 100 * k
        ws.append(W.Workload(d.name, d, W.gen_stimulus(s, d, T), W.gen_faults(s, d, 1500), T))
    refs = [oracle.fault_sim(w.design, w.stimulus, w.T, w.faults) for w in ws]
    ds, gs = _load(ws)
    prios = [np.log2(1 + r[1].astype(np.float32)) for r in refs]
    b = riros.Batch(ds, gs, [w.faults for w in ws], prios, theta=float(np.quantile(np.concatenate(prios), 0.95)),
                    monitor_rate=2.0, unified=1, struct_share=2, heavy_wg=128, light_cap=4, xcd_queues=1,
                    lockstep=1)
    for rep in range(2):
        b.launch()
        for i in range(len(ws)):
            det, ev, _ = b.read(i)
            np.testing.assert_array_equal(det, refs[i][0], err_msg=f"replay {rep} design {i}")
            np.testing.assert_array_equal(ev, refs[i][1], err_msg=f"replay {rep} design {i}")
    b.close()
