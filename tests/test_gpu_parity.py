"""GPU parity: the HIP path against the CPU oracle, bit-exact.

Golden traces, detect cycles, event counts and the byte-model words must be
identical to the oracle's on the same seeded inputs.  Runs on an MI355X only.
"""
import numpy as np
import pytest

import oracle
from helpers import Builder, all_faults, all_flip_faults, faults
from paper_2508_16376_amd import riros
from paper_2508_16376_amd import workloads as W

pytestmark = pytest.mark.gpu
UND = riros.UNDETECTED
MODES = [pytest.param(riros.MODE_PLAIN, id="plain"), pytest.param(riros.MODE_TWO_D, id="two_d"),
         pytest.param(riros.MODE_CONCURRENT, id="concurrent")]


def _run(design_np, stim, T, fl, mode=riros.MODE_PLAIN, drop=True, words_out=None, **kw):
    d = riros.Design(design_np)
    g = riros.Golden(d, stim, T)
    det, ev, cov = riros.fault_sim(d, g, fl, mode=mode, drop=drop, words_out=words_out, **kw)
    return det, ev, cov, d, g


def _check(design_np, stim, T, fl, mode=riros.MODE_PLAIN, drop=True, variant=1, **kw):
    print(f"[parity] design={design_np.name} N={design_np.num_nodes} T={T} F={fl.size} mode={mode} "
          f"drop={drop}", flush=True)
    words = np.empty(fl.size, dtype=np.uint64)
    det, ev, cov, d, g = _run(design_np, stim, T, fl, mode, drop, words_out=words, **kw)
    odet, oev, owords, _ = oracle.fault_sim_stats(design_np, stim, T, fl, drop=drop, variant=variant)
    np.testing.assert_array_equal(det, odet)
    np.testing.assert_array_equal(ev, oev)
    np.testing.assert_array_equal(words, owords)
    assert cov["total"] == fl.size
    assert cov["detected"] == int((odet != UND).sum())
    assert cov["fault_cycles"] == oracle.fault_cycles(odet, T)
    assert cov["events"] == int(oev.sum())
    assert cov["words"] == int(owords.sum())
    return det, ev


@pytest.fixture(scope="module")
def tiny():
    return W.tiny()


@pytest.fixture(scope="module")
def small():
    return W.medium(seed=777, F=4000, T=300, n_nodes=3000)


def test_golden_matches_oracle(tiny, small):
    for w in (tiny, small):
        d = riros.Design(w.design)
        g = riros.Golden(d, w.stimulus, w.T)
        np.testing.assert_array_equal(g.read(), oracle.golden(w.design, w.stimulus, w.T))


def test_golden_by_parts_and_whole_design():
    """Golden traces of a template design (its components packed into
    hundreds of parts, one workgroup each, values in LDS), of a layered
    design with one component larger than a part (one workgroup for the whole
    design), and of the heavy-tailed design (100,000 nodes in 1,024 parts)
    against the oracle's, every node and cycle."""
    cases = []
    d = W.gen_templates(515151, n_nodes=3000, name="tmpl")
    cases.append((d, W.gen_stimulus(515151, d, 300), 300))
    w = W.medium(seed=919, F=10, T=120, n_nodes=6000)
    cases.append((w.design, w.stimulus, w.T))
    w = W.heavy_tailed()
    cases.append((w.design, w.stimulus, 64))
    for design, stim, T in cases:
        print(f"[golden] {design.name} N={design.num_nodes} T={T}", flush=True)
        dd = riros.Design(design)
        g = riros.Golden(dd, stim, T)
        np.testing.assert_array_equal(g.read(), oracle.golden(design, stim, T), err_msg=design.name)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("drop", [True, False])
def test_tiny_full(tiny, mode, drop):
    _check(tiny.design, tiny.stimulus, tiny.T, tiny.faults, mode, drop, variant=0)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("drop", [True, False])
def test_small_layered_full(small, mode, drop):
    _check(small.design, small.stimulus, small.T, small.faults, mode, drop)


@pytest.mark.parametrize("mode", MODES)
def test_medium_full_size(mode):
    """The medium workload at its full size; every fault compared with the oracle."""
    w = W.medium()
    _check(w.design, w.stimulus, w.T, w.faults, mode, True)


def _edge_design():
    b = Builder()
    a = b.pi(64)
    c = b.pi(1)
    k = b.const(64, 0xDEADBEEF12345678)
    r64 = b.reg(64, init=0x8000000000000001)
    r1 = b.reg(1, init=1)
    s = b.node(W.ADD, 64, (a, r64))
    x = b.node(W.XOR, 64, (s, k))
    sh = b.node(W.SHL, 64, (x,), 63)
    sr = b.node(W.SHR, 64, (x,), 64)
    m = b.node(W.MUX, 64, (r1, x, sh))
    cc = b.node(W.CONCAT, 64, (b.node(W.SLICE, 32, (m,), 16), b.node(W.SLICE, 32, (a,), 32)))
    lt = b.node(W.ULT, 1, (cc, x))
    nt = b.node(W.NOT, 1, (lt,))
    ml = b.node(W.MUL, 64, (cc, a))
    b.set_d(r64, ml)
    b.set_d(r1, b.node(W.XOR, 1, (nt, c)))
    eq = b.node(W.EQ, 1, (sr, b.const(64, 0)))
    return b.design([nt, cc, eq, r1], "edge64")


@pytest.mark.parametrize("mode", MODES)
def test_edge_design_all_faults_all_sites(mode):
    d = _edge_design()
    T = 150
    stim = W.counter_values(99, 0, 2 * T).reshape(T, 2)
    stim[:, 1] &= np.uint64(1)
    fl = all_faults(d)                     # includes PI, CONST, REG and output nodes
    for drop in (True, False):
        _check(d, stim, T, fl, mode, drop, variant=0)


@pytest.mark.parametrize("mode", MODES)
def test_single_cycle_single_fault_and_duplicates(tiny, mode):
    w = tiny
    _check(w.design, w.stimulus, 1, w.faults[:1], mode)
    dup = np.concatenate([w.faults[:50], w.faults[:50]])
    det, ev = _check(w.design, w.stimulus, w.T, dup, mode)
    np.testing.assert_array_equal(det[:50], det[50:])


@pytest.mark.parametrize("mode", MODES)
def test_no_registers_and_register_chain(mode):
    b = Builder()
    p = [b.pi(8) for _ in range(3)]
    o = b.node(W.SUB, 8, (b.node(W.AND, 8, (p[0], p[1])), p[2]))
    d = b.design([o], "comb-only")
    T = 64
    stim = W.counter_values(3, 0, 3 * T).reshape(T, 3) & np.uint64(255)
    _check(d, stim, T, all_faults(d), mode, variant=0)
    b = Builder()
    x = b.pi(4)
    regs = [b.reg(4) for _ in range(6)]
    b.set_d(regs[0], x)
    for j in range(1, 6):
        b.set_d(regs[j], regs[j - 1])
    d = b.design([regs[-1]], "delay-line")
    stim = (W.counter_values(4, 0, T) & np.uint64(15))[:, None]
    _check(d, stim, T, all_faults(d), mode, variant=0)


@pytest.mark.parametrize("mode", MODES)
def test_faults_in_any_order_give_the_same_results(small, mode):
    w = small
    perm = np.argsort(W.counter_values(5, 0, w.faults.size))
    det, ev, _, _, _ = _run(w.design, w.stimulus, w.T, w.faults, mode)
    det2, ev2, _, _, _ = _run(w.design, w.stimulus, w.T, w.faults[perm], mode)
    np.testing.assert_array_equal(det[perm], det2)
    np.testing.assert_array_equal(ev[perm], ev2)


def test_repeated_calls_reuse_workspace(small):
    """Stamps carry over between calls on one design handle; results must not."""
    w = small
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    first = riros.fault_sim(d, g, w.faults)
    for wpc, mode in ((1, 0), (4, 1), (16, 0), (2, 1)):
        again = riros.fault_sim(d, g, w.faults, waves_per_cu=wpc, mode=mode)
        np.testing.assert_array_equal(first[0], again[0])
        np.testing.assert_array_equal(first[1], again[1])


def test_invalid_fault_rejected(tiny):
    d = riros.Design(tiny.design)
    g = riros.Golden(d, tiny.stimulus, tiny.T)
    bad = tiny.faults[:4].copy()
    bad["bit"][2] = 70
    with pytest.raises(riros.RirosError) as e:
        riros.fault_sim(d, g, bad)
    assert e.value.code == riros.RIROS_EINVAL
    bad = tiny.faults[:4].copy()
    bad["site"][1] = tiny.design.num_nodes
    with pytest.raises(riros.RirosError):
        riros.fault_sim(d, g, bad)


def test_empty_fault_list(tiny):
    d = riros.Design(tiny.design)
    g = riros.Golden(d, tiny.stimulus, tiny.T)
    det, ev, cov = riros.fault_sim(d, g, tiny.faults[:0])
    assert det.size == 0 and cov["total"] == 0


def test_device_io_matches_host_io(small):
    import torch
    w = small
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    det, ev, cov = riros.fault_sim(d, g, w.faults)
    dev = torch.device("cuda:0")
    f_dev = torch.from_numpy(w.faults.view(np.uint8).copy()).to(dev)
    det_dev = torch.empty(w.faults.size, dtype=torch.int32, device=dev)
    ev_dev = torch.empty(w.faults.size, dtype=torch.int64, device=dev)
    cov_dev = torch.zeros(riros.COVERAGE_FIELDS, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    opts = riros.make_opts(riros.MODE_PLAIN, True, True, stream=stream)
    riros.fault_sim_device(d, g, f_dev, w.faults.size, det_dev, ev_dev, cov_dev, opts)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(det_dev.cpu().numpy().view(np.uint32), det)
    np.testing.assert_array_equal(ev_dev.cpu().numpy().view(np.uint64), ev)
    c = cov_dev.cpu().numpy()
    assert list(c) == [cov["detected"], cov["total"], cov["fault_cycles"], cov["events"], cov["words"]]


@pytest.mark.parametrize("light_cap", [4, 8, 16])
def test_two_d_light_capacity_does_not_change_results(small, light_cap):
    """Smaller capacities hand more faults to the heavy path; results are identical."""
    _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, True, light_cap=light_cap)


@pytest.mark.parametrize("theta", [float("-inf"), 0.25, 0.5, 0.9, float("inf")])
def test_two_d_priority_and_threshold(small, theta):
    """Random priorities: any order and any light/heavy split give identical results."""
    prio = (W.counter_values(11, 0, small.faults.size) >> np.uint64(40)).astype(np.float32) / np.float32(1 << 24)
    for drop in (True, False):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop,
               priority=prio, theta=theta)


@pytest.mark.parametrize("rate", [0.5, 2.0, 8.0])
def test_two_d_monitor_hand_over(small, rate):
    """The events-per-cycle monitor moves faults to the structural path; results are identical."""
    for drop in (True, False):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, monitor_rate=rate)


@pytest.mark.parametrize("rate", [0.5, 4.0])
@pytest.mark.parametrize("light_cap", [4, 8])
def test_two_d_unified_schedule(small, rate, light_cap):
    """Launch-A wavefronts that run out of light work take handed-over faults
    while others still run light work; results are identical."""
    for drop in (True, False):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, monitor_rate=rate,
               light_cap=light_cap, unified=1)


def test_two_d_unified_with_heavy_prefix_and_small_grid(small):
    prio = (W.counter_values(12, 0, small.faults.size) >> np.uint64(40)).astype(np.float32) / np.float32(1 << 24)
    for wpc in (1, 4):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, True, priority=prio,
               theta=0.9, monitor_rate=1.0, unified=1, waves_per_cu=wpc)


@pytest.mark.parametrize("share", [1, 2, 4])
def test_two_d_shared_structural_workspace(small, share):
    """Launch-A workgroups of 1, 2 or 4 wavefronts share one structural
    workspace (only the first takes structural work); with a heavy prefix,
    the unified schedule and the monitor, results are identical."""
    prio = (W.counter_values(13, 0, small.faults.size) >> np.uint64(40)).astype(np.float32) / np.float32(1 << 24)
    for unified, theta in ((1, 0.8), (0, 0.5), (1, float("inf"))):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, True, priority=prio,
               theta=theta, monitor_rate=1.0, unified=unified, struct_share=share)
    for wpc in (1, 5):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, False, priority=prio,
               theta=0.9, monitor_rate=2.0, unified=1, struct_share=share, waves_per_cu=wpc)


@pytest.mark.parametrize("heavy_wg", [128, 256])
def test_two_d_workgroup_structural_split(small, tiny, heavy_wg):
    """A structural fault simulated by 2 or 4 wavefronts (the frontier of
    each pass split across all their lanes, one barrier per pass): in launch
    B for handed-over faults, and in launch A's heavy prefix when its
    workgroups hold several wavefronts; drop on and off, every fault on the
    structural path (theta -inf) or a prefix of them, small grids."""
    prio = (W.counter_values(17, 0, small.faults.size) >> np.uint64(40)).astype(np.float32) / np.float32(1 << 24)
    for drop in (True, False):
        for share, theta, unified in ((1, float("inf"), 0), (2, float("-inf"), 0), (4, 0.7, 1), (2, 0.5, 1)):
            _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, priority=prio,
                   theta=theta, monitor_rate=1.0, light_cap=4, unified=unified, struct_share=share,
                   heavy_wg=heavy_wg)
    _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, True, priority=prio,
           theta=0.5, monitor_rate=0.5, unified=0, struct_share=4, heavy_wg=heavy_wg, waves_per_cu=1)
    tp = np.ones(tiny.faults.size, dtype=np.float32)
    _check(tiny.design, tiny.stimulus, tiny.T, tiny.faults, riros.MODE_TWO_D, False, priority=tp,
           theta=0.0, struct_share=4, heavy_wg=heavy_wg)


def test_two_d_workgroup_split_medium_no_drop_sample():
    """Dense faults (no dropping, the paper's convention): every fault of a
    sample of the medium list on four-wavefront structural workgroups."""
    w = W.medium()
    idx = np.sort(np.argsort(W.counter_values(0xD0D0, 0, w.faults.size), kind="stable")[:100])
    prio = np.ones(idx.size, dtype=np.float32)
    _check(w.design, w.stimulus, w.T, w.faults[idx], riros.MODE_TWO_D, False, priority=prio, theta=0.0,
           struct_share=4, heavy_wg=256, unified=1)
    _check(w.design, w.stimulus, w.T, w.faults[idx], riros.MODE_TWO_D, False, light_cap=4, monitor_rate=0.5,
           heavy_wg=256)


@pytest.mark.parametrize("light_cap", [4, 8])
def test_two_d_lockstep_lanes(small, tiny, light_cap):
    """Light lanes that start their cycles together (lockstep), with and
    without priorities (faults of one site adjacent), drop on and off."""
    prio = (W.counter_values(19, 0, small.faults.size) >> np.uint64(52)).astype(np.float32)
    for drop in (True, False):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, lockstep=1,
               light_cap=light_cap, monitor_rate=2.0)
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, lockstep=1,
               light_cap=light_cap, priority=prio, unified=1, monitor_rate=1.0)
    _check(tiny.design, tiny.stimulus, tiny.T, tiny.faults, riros.MODE_TWO_D, False, lockstep=1, light_cap=light_cap)


@pytest.mark.parametrize("deal", [4, 8, 32])
def test_two_d_dealt_light_queue(small, tiny, deal):
    """The head of the light queue dealt out in groups over every wavefront:
    one wavefront per compute unit (256 rows of 64 positions, fewer than the
    4,000 faults: the deal covers part of the queue) and twelve (the queue
    ends inside the dealt rows), with and without priorities, lockstep on and
    off, drop on and off."""
    prio = (W.counter_values(23, 0, small.faults.size) >> np.uint64(50)).astype(np.float32)
    for drop in (True, False):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, deal=deal,
               waves_per_cu=1, light_cap=4, lockstep=1, priority=prio, unified=1)
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, deal=deal,
               waves_per_cu=12, light_cap=8, monitor_rate=2.0)
    _check(tiny.design, tiny.stimulus, tiny.T, tiny.faults, riros.MODE_TWO_D, True, deal=deal, lockstep=1)


@pytest.mark.parametrize("head_lanes", [1, 16, 40])
def test_two_d_head_batch(small, tiny, head_lanes):
    """A wavefront's first take limited to head_lanes faults, finished before
    it takes more; with priorities, lockstep and a dealt head, drop on and
    off, one and twelve wavefronts per compute unit."""
    prio = (W.counter_values(31, 0, small.faults.size) >> np.uint64(50)).astype(np.float32)
    for drop in (True, False):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, head_lanes=head_lanes,
               waves_per_cu=1, light_cap=4, lockstep=1, priority=prio, unified=1, struct_share=4)
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, head_lanes=head_lanes,
               deal=8, waves_per_cu=12, light_cap=8, monitor_rate=2.0, priority=prio)
    _check(tiny.design, tiny.stimulus, tiny.T, tiny.faults, riros.MODE_TWO_D, True, head_lanes=head_lanes)


@pytest.mark.parametrize("light_cap", [4, 8])
def test_two_d_xcd_queues(small, tiny, light_cap):
    """Per-XCD light queues: the priority order partitioned by the site's XCD,
    each wavefront taking its own XCD's part first and then the others'; with
    a heavy prefix, lockstep, a head batch, one and twelve wavefronts per
    compute unit, drop on and off; without priorities the option changes
    nothing."""
    prio = (W.counter_values(37, 0, small.faults.size) >> np.uint64(50)).astype(np.float32)
    for drop in (True, False):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, xcd_queues=1,
               waves_per_cu=1, light_cap=light_cap, lockstep=1, priority=prio, unified=1, struct_share=4)
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, drop, xcd_queues=1,
               waves_per_cu=12, light_cap=light_cap, monitor_rate=2.0, priority=prio,
               theta=float(np.quantile(prio, 0.95)), head_lanes=16)
    _check(small.design, small.stimulus, small.T, small.faults[:700], riros.MODE_TWO_D, True, xcd_queues=1,
           light_cap=light_cap)
    _check(tiny.design, tiny.stimulus, tiny.T, tiny.faults, riros.MODE_TWO_D, True, xcd_queues=1,
           priority=np.ones(tiny.faults.size, np.float32), light_cap=light_cap)


@pytest.mark.parametrize("drop", [True, False])
def test_two_d_32bit_lanes_template_design(drop):
    """A template design (every node at most 32 bits wide: the light lanes
    keep 32-bit values, evaluate two nodes per iteration and cache the
    register they last evaluated, also when it is the fault site), all of its
    faults and flips, under several schedules."""
    d = W.gen_templates(252525, n_nodes=4000, name="tmpl32")
    T = 400
    stim = W.gen_stimulus(252525, d, T)
    fl = W.gen_faults(252525, d, 6000)
    flips = W.gen_flip_faults(252526, d, 1500, T)
    prio = (W.counter_values(41, 0, fl.size) >> np.uint64(50)).astype(np.float32)
    for kw in ({"light_cap": 4, "lockstep": 1, "priority": prio},
               {"light_cap": 4, "lockstep": 0, "unified": 1, "struct_share": 4, "priority": prio},
               {"light_cap": 4, "lockstep": 1, "waves_per_cu": 1},
               {"light_cap": 8, "lockstep": 1, "priority": prio, "monitor_rate": 2.0}):
        _check(d, stim, T, fl, riros.MODE_TWO_D, drop, **kw)
    _check(d, stim, T, flips, riros.MODE_TWO_D, drop, light_cap=4, lockstep=1)


@pytest.mark.parametrize("drop", [True, False])
def test_two_d_tuned_schedules_template_design(drop):
    """The schedules the autotuner picks on the template workloads: head
    batches filling all 64 lanes, free-running lanes, the unified schedule
    with the monitor off and workspaces shared by four wavefronts, and
    (without dropping) capacity 8; every fault against the oracle."""
    d = W.gen_templates(262626, n_nodes=6000, name="tmpl_tuned")
    T = 600
    stim = W.gen_stimulus(262626, d, T)
    fl = W.gen_faults(262626, d, 8000)
    prio = (W.counter_values(43, 0, fl.size) >> np.uint64(50)).astype(np.float32)
    base = {"lockstep": 0, "head_lanes": 64, "waves_per_cu": 16, "heavy_wg": 64, "priority": prio}
    for kw in ({"light_cap": 4, "unified": 0, "monitor_rate": 4.0, "struct_share": 2},
               {"light_cap": 4, "unified": 1, "monitor_rate": 0.0, "struct_share": 4},
               {"light_cap": 8, "unified": 1, "monitor_rate": 0.0, "struct_share": 4}):
        _check(d, stim, T, fl, riros.MODE_TWO_D, drop, **base, **kw)


def test_two_d_dealt_medium_full_size():
    """50,000 faults over 256 wavefronts: 16,384 dealt positions, then the rest
    of the queue in order."""
    w = W.medium()
    prio = (W.counter_values(29, 0, w.faults.size) >> np.uint64(48)).astype(np.float32)
    _check(w.design, w.stimulus, w.T, w.faults, riros.MODE_TWO_D, True, deal=8, waves_per_cu=1, light_cap=4,
           lockstep=1, unified=1, struct_share=4, priority=prio)


def test_two_d_unified_medium_full_size():
    w = W.medium()
    _check(w.design, w.stimulus, w.T, w.faults, riros.MODE_TWO_D, True, monitor_rate=2.0, light_cap=4, unified=1)


def test_two_d_rejects_bad_options(tiny):
    d = riros.Design(tiny.design)
    g = riros.Golden(d, tiny.stimulus, tiny.T)
    for kw in ({"unified": 2}, {"monitor_rate": -1.0}, {"light_cap": 5}, {"struct_share": 3}, {"struct_share": 8},
               {"heavy_wg": 96}, {"heavy_wg": 512}, {"deal": 2}, {"deal": 12}, {"deal": 64},
               {"head_lanes": -1}, {"head_lanes": 65}, {"xcd_queues": 2},
               {"lockstep": 2}):
        with pytest.raises(riros.RirosError):
            riros.fault_sim(d, g, tiny.faults[:10], mode=riros.MODE_TWO_D, **kw)


@pytest.mark.parametrize("mode", MODES)
def test_narrow_schedule_passes(small, mode):
    """32 wavefronts per compute unit make the structural LDS take the narrow
    pass (16 schedule words, a 2 KB list); dense levels (no dropping) then
    take several passes.  Results are identical."""
    for drop in (True, False):
        _check(small.design, small.stimulus, small.T, small.faults[:1500], mode, drop, waves_per_cu=32,
               **({} if mode == riros.MODE_PLAIN else {"unified": 1, "monitor_rate": 1.0, "light_cap": 4}))


def test_two_d_waves_per_cu(small):
    for wpc in (1, 3):
        _check(small.design, small.stimulus, small.T, small.faults, riros.MODE_TWO_D, True, waves_per_cu=wpc)


def test_two_d_device_io_with_priority(small):
    import torch
    w = small
    d = riros.Design(w.design)
    g = riros.Golden(d, w.stimulus, w.T)
    det, ev, cov = riros.fault_sim(d, g, w.faults)
    dev = torch.device("cuda:0")
    prio = torch.from_numpy((np.arange(w.faults.size) % 97).astype(np.float32)).to(dev)
    f_dev = torch.from_numpy(w.faults.view(np.uint8).copy()).to(dev)
    det_dev = torch.empty(w.faults.size, dtype=torch.int32, device=dev)
    ev_dev = torch.empty(w.faults.size, dtype=torch.int64, device=dev)
    cov_dev = torch.zeros(riros.COVERAGE_FIELDS, dtype=torch.int64, device=dev)
    opts = riros.make_opts(riros.MODE_TWO_D, True, True, stream=torch.cuda.current_stream(), priority=prio,
                           theta=90.0)
    riros.fault_sim_device(d, g, f_dev, w.faults.size, det_dev, ev_dev, cov_dev, opts)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(det_dev.cpu().numpy().view(np.uint32), det)
    np.testing.assert_array_equal(ev_dev.cpu().numpy().view(np.uint64), ev)


# ---------------------------------------------------------------------------
# Bit flips (transient faults): the same paths, a different faulty-value rule
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("drop", [True, False])
def test_flips_tiny_every_site_bit_and_cycle_window(tiny, mode, drop):
    """A flip on every bit of every node, in cycles 0, 1, 63, 64 and the last."""
    w = tiny
    fl = all_flip_faults(w.design, 1)
    rows = []
    for t0 in (0, 1, 63, 64, w.T - 1, w.T):
        f = fl.copy()
        f["t0"] = t0
        rows.append(f)
    fl = np.concatenate(rows)
    _check(w.design, w.stimulus, w.T, fl, mode, drop, variant=0)


@pytest.mark.parametrize("kw", [{"mode": riros.MODE_PLAIN}, {"mode": riros.MODE_TWO_D},
                                {"mode": riros.MODE_TWO_D, "monitor_rate": 1.0, "unified": 1},
                                {"mode": riros.MODE_TWO_D, "light_cap": 4, "monitor_rate": 0.5},
                                {"mode": riros.MODE_CONCURRENT}],
                         ids=["plain", "two_d", "two_d_unified", "two_d_cap4", "concurrent"])
def test_flips_and_stuck_mixed_small(small, kw):
    w = small
    fl = np.concatenate([w.faults[:2000], W.gen_flip_faults(17, w.design, 3000, w.T + 30)])
    perm = np.argsort(W.counter_values(18, 0, fl.size))
    fl = fl[perm]
    kw = dict(kw)
    mode = kw.pop("mode")
    for drop in (True, False):
        _check(w.design, w.stimulus, w.T, fl, mode, drop, **kw)


@pytest.mark.parametrize("mode", MODES)
def test_flips_medium_full_size(mode):
    """50,000 flips on the medium design, every one compared with the oracle."""
    w = W.medium()
    fl = W.gen_flip_faults(19, w.design, 50000, w.T)
    _check(w.design, w.stimulus, w.T, fl, mode, True, unified=1 if mode == riros.MODE_TWO_D else 0,
           monitor_rate=2.0 if mode == riros.MODE_TWO_D else 0.0)
