"""Fault-simulation throughput benchmark (fault-cycles per second) on one GPU.

One step = one pass of the whole hot path over the workload's fault list with
inputs (design image, golden trace, fault list, predicted priorities) already
resident in device memory: riros_fault_sim for one design, one campaign
graph launch for the batched campaign.  Fault-cycles per fault are
detect cycle + 1, or the cycle count if undetected.  Prints one JSON line.

The default workload is the large one (200,000-node template design, 10,000
cycles, 1,000,000 stuck-at faults), scheduled by the load predictor and the
autotuner; the line also carries the plain kernel on the same list, the
ablation ladder, and the 64-design batched campaign as a second measured leg
(plain per-design kernels against one predictor-ordered graph launch).

    python bench.py [--steps K] [--warmup W] [--workload large|heavy_tailed|medium|tiny|campaign]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2508_16376_amd import autotune, predictor, riros  # noqa: E402
from paper_2508_16376_amd import workloads as W  # noqa: E402

# Published MI355X peaks: HBM3E 8 TB/s.  The int32 vector-ALU peak follows
# from the published 157.3 TFLOP/s FP32 vector rate, 256 compute units x 128
# lanes a clock x 2 flops (an FMA) x 2.4 GHz: 128 single-cycle int32 lane
# operations a clock per compute unit (the probe measures about 70% of it).
HBM_PEAK_GBS = 8000.0
VALU_PEAK_OPS = 256 * 128 * 2.4e9
# Bytes of the byte model: 4 per word (riros_sim_opts.words counts the words
# each fault must touch: its site's golden word per simulated cycle, k + 2
# per event at a node with k operands, 2 more per divergent register, every
# word twice for nodes wider than 32 bits).
BYTES_PER_WORD = 4
# Algorithmic integer operations: about 10 per event (input selects, the
# operator, the compare with the golden value, scheduling the users) and 3
# per fault-cycle (the excitation check).
OPS_PER_EVENT = 10
OPS_PER_FC = 3
NO_DROP_SAMPLE = 20000     # faults of the no-dropping leg (seeded draw)
NO_DROP_PROBE = 2000       # its first faults, timed first to bound the leg
NO_DROP_MAX_MS = 3000.0    # a pass of the full sample longer than this keeps the probe
NO_DROP_PROBE_TUNE_MS = 2000.0   # the probe is tuned when its pass takes at most this
NO_DROP_TUNE_BUDGET_S = 20.0
# in the order descended: the two that move the most first, so that a design
# whose candidates take seconds reaches them within the budget
NO_DROP_TUNED = ("light_cap", "heavy_wg", "unified", "monitor_rate")
TRAIN_EPOCHS = 30
PLAIN_STEPS = 2          # the plain kernel is timed on at most this many steps
TUNE_BUDGET_S = 45.0
CAMPAIGN_TUNE_BUDGET_S = 30.0
TUNE_SAMPLE = 250000     # faults the tuner times each candidate on (seeded draw)

WORKLOADS = {
    "tiny": "tiny: 144-node DAG (120 operators, 16 registers), 128 cycles, 2,000 stuck-at faults",
    "medium": "medium: 20,000-node layered DAG (40 levels, 512 registers, widths 1-64), 1,000 cycles, "
              "50,000 stuck-at faults, drop on",
    "heavy_tailed": "heavy-tailed: 100,000-node template design (pipelines, 8-bit FSMs, latent 32-bit "
                    "accumulators), 5,000 cycles, 200,000 stuck-at faults",
    "campaign": "batched campaign: 64 seeded designs (1k-50k nodes log-uniform, 3-10% registers), "
                "1k-100k faults each (log-uniform), 500-5,000 cycles each, one graph launch",
    "large": "large: 200,000-node template design (config-2 style), 10,000 cycles, 1,000,000 stuck-at "
             "faults, predictor-scheduled",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_digest():
    """Digest of the HIP sources; a counter summary taken on other sources no
    longer describes the kernels that run."""
    h = hashlib.sha1()
    src = os.path.join(ROOT, "paper_2508_16376_amd", "csrc")
    for name in sorted(os.listdir(src)):
        with open(os.path.join(src, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per fault-simulation pass (FETCH_SIZE and WRITE_SIZE counters,
    each scaled by the same counter's reading for a copy of known size), from
    the committed counter summary of this workload; None when there is none or
    it was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            m = re.match(r"^- (\w+): `?([^`\s]+)`?", line)
            if m:
                fields[m.group(1)] = m.group(2)
    if fields.get("kernel_sources") != kernel_source_digest() or "hbm_bytes_per_pass" not in fields:
        return None
    return float(fields["hbm_bytes_per_pass"])


def no_drop_sample(F, probe_n, probe_ms):
    """Faults of the no-dropping leg and whether to tune it: the full sample
    (NO_DROP_SAMPLE faults, or the whole list if shorter), tuned, unless its
    pass, extrapolated from the probe's, would exceed NO_DROP_MAX_MS; then the
    probe's faults, tuned only if a probe pass takes at most
    NO_DROP_PROBE_TUNE_MS (each candidate is timed three times)."""
    n = min(F, NO_DROP_SAMPLE)
    if probe_n <= 0 or probe_ms * n / probe_n > NO_DROP_MAX_MS:
        return probe_n, probe_n > 0 and probe_ms <= NO_DROP_PROBE_TUNE_MS
    return n, True


COPY_BYTES = 1 << 30


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def copy_calibration():
    """One device-to-device copy of COPY_BYTES bytes (read COPY_BYTES, write
    COPY_BYTES): the known-size reference for the HBM byte counters."""
    import torch
    src = torch.full((COPY_BYTES // 8,), 7, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    assert int(dst[-1]) == 7
    print(json.dumps({"copy_bytes": COPY_BYTES}))


def make_workload(name):
    if name == "tiny":
        return [W.tiny()]
    if name == "medium":
        return [W.medium()]
    if name == "heavy_tailed":
        return [W.heavy_tailed()]
    if name == "large":
        return [W.large()]
    return W.campaign()


def held_out_training_runs():
    """Designs of the medium, heavy-tailed (at 1,000, 5,000 and 10,000 cycles)
    and campaign shapes with seeds other than any benchmark workload; their
    plain-kernel event counts train the predictor."""
    ws = [W.medium(seed=7001, F=20000, T=1000), W.medium(seed=7002, F=20000, T=1000),
          W.heavy_tailed(seed=7003, F=20000, T=1000, n_nodes=30000),
          W.heavy_tailed(seed=7005, F=30000, T=5000, n_nodes=30000),
          W.heavy_tailed(seed=7006, F=30000, T=10000, n_nodes=40000)]
    ws += W.campaign(seed=7004, n=6, nodes=(1000, 20000), faults=(2000, 10000), cycles=(500, 2000))
    runs = []
    for w in ws:
        d = riros.Design(w.design)
        runs.append((d, riros.Golden(d, w.stimulus, w.T), w.faults))
    return runs


class Single:
    """One design: steps are riros_fault_sim calls with device-resident I/O."""

    def __init__(self, w):
        import torch
        self.w = w
        self.d = riros.Design(w.design)
        torch.cuda.synchronize()
        t = time.perf_counter()
        self.g = riros.Golden(self.d, w.stimulus, w.T)
        self.golden_s = time.perf_counter() - t
        dev = torch.device("cuda:0")
        F = w.faults.size
        self.F = F
        self.f_dev = torch.from_numpy(w.faults.view(np.uint8).copy()).to(dev)
        self.det = torch.empty(F, dtype=torch.int32, device=dev)
        self.ev = torch.empty(F, dtype=torch.int64, device=dev)
        self.wk = torch.empty(F, dtype=torch.int64, device=dev)
        self.cov = torch.zeros(riros.COVERAGE_FIELDS, dtype=torch.int64, device=dev)
        self.prio_dev = None

    def features(self):
        return riros.features(self.d, self.g, self.w.faults)

    def set_priority(self, pred):
        import torch
        self.prio_dev = None if pred is None else torch.from_numpy(np.ascontiguousarray(pred, np.float32)).cuda()

    def run(self, mode, steps, warmup, kw, drop=True):
        import torch
        opts = riros.make_opts(mode, drop, True, stream=torch.cuda.current_stream(),
                               priority=self.prio_dev if mode == riros.MODE_TWO_D else None, words=self.wk, **kw)
        for _ in range(warmup):
            riros.fault_sim_device(self.d, self.g, self.f_dev, self.F, self.det, self.ev, self.cov, opts)
        torch.cuda.synchronize()
        kms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            riros.fault_sim_device(self.d, self.g, self.f_dev, self.F, self.det, self.ev, self.cov, opts)
            kms.append(riros.last_kernel_ms())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        c = self.cov.cpu().numpy().astype(np.int64)
        return {"wall_s": wall, "steps": steps, "kernel_ms": float(np.mean(kms)), "fault_cycles": int(c[2]),
                "events": int(c[3]), "words": int(c[4]), "detected": int(c[0]),
                "detect": [self.det.cpu().numpy().view(np.uint32).copy()],
                "events_arr": [self.ev.cpu().numpy().view(np.uint64).copy()],
                "words_arr": [self.wk.cpu().numpy().view(np.uint64).copy()]}


class Campaign:
    """Many designs: a plain step runs riros_fault_sim per design; a batched
    step is one graph launch of the whole campaign."""

    def __init__(self, ws):
        import torch
        self.ws = ws
        self.ds = [riros.Design(w.design) for w in ws]
        torch.cuda.synchronize()
        t = time.perf_counter()
        self.gs = riros.Golden.many(self.ds, [w.stimulus for w in ws], [w.T for w in ws])
        self.golden_s = time.perf_counter() - t

    def features(self):
        return [riros.features(d, g, w.faults) for d, g, w in zip(self.ds, self.gs, self.ws)]

    def run_plain(self, steps, warmup):
        import torch
        for _ in range(warmup):
            for d, g, w in zip(self.ds, self.gs, self.ws):
                riros.fault_sim(d, g, w.faults, mode=riros.MODE_PLAIN)
        kms, res = [], None
        t0 = time.perf_counter()
        for _ in range(steps):
            k = 0.0
            res = []
            for d, g, w in zip(self.ds, self.gs, self.ws):
                res.append(riros.fault_sim(d, g, w.faults, mode=riros.MODE_PLAIN))
                k += riros.last_kernel_ms()
            kms.append(k)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # a plain step includes host-side fault upload and result download per
        # design; its rate uses the summed kernel time instead of the wall
        return {"wall_s": wall, "steps": steps, "kernel_ms": float(np.mean(kms)), "kernel_bound": True,
                "fault_cycles": sum(r[2]["fault_cycles"] for r in res), "events": sum(r[2]["events"] for r in res),
                "words": sum(r[2]["words"] for r in res),
                "detected": sum(r[2]["detected"] for r in res), "detect": [r[0] for r in res],
                "events_arr": [r[1] for r in res]}

    def run_batch(self, steps, warmup, kw, prios, drop=True):
        import torch
        b = riros.Batch(self.ds, self.gs, [w.faults for w in self.ws], prios, drop=drop, **kw)
        s = torch.cuda.current_stream()
        for _ in range(warmup):
            b.launch(s)
        torch.cuda.synchronize()
        kms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            b.launch(s)
            kms.append(riros.last_kernel_ms())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        res = [b.read(i) for i in range(len(self.ws))]
        b.close()
        return {"wall_s": wall, "steps": steps, "kernel_ms": float(np.mean(kms)),
                "fault_cycles": sum(r[2]["fault_cycles"] for r in res), "events": sum(r[2]["events"] for r in res),
                "words": sum(r[2]["words"] for r in res),
                "detected": sum(r[2]["detected"] for r in res), "detect": [r[0] for r in res],
                "events_arr": [r[1] for r in res]}


def rate(r):
    if r.get("kernel_bound"):
        return r["fault_cycles"] / (r["kernel_ms"] * 1e-3)
    return r["fault_cycles"] * r["steps"] / r["wall_s"]


def same_results(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a["detect"], b["detect"])) and \
        all(np.array_equal(x, y) for x, y in zip(a["events_arr"], b["events_arr"]))


def train_predictor():
    t = time.perf_counter()
    runs = held_out_training_runs()
    x, y = predictor.samples_from_runs(runs)
    data_s = time.perf_counter() - t
    t = time.perf_counter()
    wts, losses = predictor.train(x, y, epochs=TRAIN_EPOCHS, batch=4096)
    train_s = time.perf_counter() - t
    del runs
    return wts, {"train_samples": int(x.shape[0]), "train_data_s": data_s, "train_s": train_s,
                 "final_loss": float(losses[-1])}


def best_single_feature(feats, true):
    """Spearman of the best single feature (either sign), the baseline the
    network has to beat."""
    best = (-1.0, None)
    for k in range(feats.shape[1]):
        rho = predictor.load_error(feats[:, k], true)["spearman"]
        for r, sgn in ((rho, 1), (-rho, -1)):
            if r > best[0]:
                best = (r, (k, sgn))
    return best


def campaign_leg(args, wts):
    """The 64-design campaign: plain per-design kernels, then one graph launch
    ordered by the predictor (the same trained weights), with schedule
    parameters tuned for the campaign (a shorter wall budget)."""
    t = time.perf_counter()
    ws = W.campaign()
    log(f"[bench] campaign: generated in {time.perf_counter() - t:.1f}s")
    job = Campaign(ws)
    log(f"[bench] campaign golden traces: {job.golden_s:.2f}s")
    plain = job.run_plain(1, 1)
    log(f"[bench] campaign plain: kernel {plain['kernel_ms']:.1f} ms, {rate(plain):.4g} FC/s")
    feats = job.features()
    preds = [riros.mlp_predict(wts, f) for f in feats] if wts is not None else None
    allp = None if preds is None else np.concatenate(preds)
    t = time.perf_counter()
    if args.no_tune:
        params = dict(autotune.DEFAULT)
    else:
        tuner = autotune.Autotuner(progress=log, budget_s=CAMPAIGN_TUNE_BUDGET_S)
        params = tuner.tune_batch([w.design for w in ws], job.ds, job.gs, [w.faults for w in ws], preds)
    tune_s = time.perf_counter() - t
    log(f"[bench] campaign autotuner: {params} in {tune_s:.1f}s")
    static = job.run_batch(2, 1, autotune.batch_kwargs(dict(params, heavy_quantile=None)), None)
    best = job.run_batch(args.steps, args.warmup, autotune.batch_kwargs(params, allp), preds)
    withg = job.run_batch(2, 1, dict(autotune.batch_kwargs(params, allp), campaign_golden=True), preds)
    log(f"[bench] campaign batched: static {static['kernel_ms']:.1f} ms, predictor {best['kernel_ms']:.1f} ms, "
        f"with golden traces in the graph {withg['kernel_ms']:.1f} ms")
    out = {"workload": WORKLOADS["campaign"], "designs": len(ws), "faults": int(sum(w.faults.size for w in ws)),
           "golden_s": job.golden_s,
           "plain": {"fault_cycles_per_s": rate(plain), "kernel_ms": plain["kernel_ms"],
                     "note": "sum of 64 per-design kernel times"},
           "batched_static": {"fault_cycles_per_s": rate(static), "kernel_ms": static["kernel_ms"]},
           "batched_predictor": {"fault_cycles_per_s": rate(best), "kernel_ms": best["kernel_ms"],
                                 "steps": best["steps"], "ms_per_step": best["wall_s"] / best["steps"] * 1e3},
           "batched_predictor_golden_in_graph": {"fault_cycles_per_s": rate(withg), "kernel_ms": withg["kernel_ms"],
                                                 "note": "each launch also recomputes the 64 golden traces"},
           "speedup_vs_plain": rate(best) / rate(plain),
           "fault_cycles": best["fault_cycles"], "events": best["events"], "words": best["words"],
           "results_identical": bool(same_results(plain, best) and same_results(static, best) and
                                     same_results(withg, best)),
           "params": params, "tune_s": tune_s}
    del job
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-predictor", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-drop-leg", choices=["on", "off"], default="on",
                    help="extra run without fault dropping (the paper's convention) on a sample of the faults")
    ap.add_argument("--concurrent-leg", choices=["on", "off"], default="on",
                    help="extra timing of the concurrent (node-major) mode on the same workload")
    ap.add_argument("--campaign-leg", choices=["on", "off"], default="on",
                    help="the 64-design batched campaign as a second measured leg (single-design workloads)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run one copy of known size (for scaling the HBM byte counters)")
    ap.add_argument("--params", default=None,
                    help="schedule parameters as JSON (the autotuner's output): no tuning")
    ap.add_argument("--only-headline", action="store_true",
                    help="run only the timed predictor leg (for kernel traces and counters: every fault-"
                         "simulation launch of the run is then one of the timed ones)")
    args = ap.parse_args()
    if args.only_headline:
        args.no_cpu_baseline = True
        args.no_drop_leg = args.concurrent_leg = args.campaign_leg = "off"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): sharding the fault list across "
              "GPUs (by fault, with one final gather) is not implemented.", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    t = time.perf_counter()
    ws = make_workload(args.workload)
    log(f"[bench] workload {args.workload}: generated in {time.perf_counter() - t:.2f}s")
    multi = args.workload == "campaign"
    job = Campaign(ws) if multi else Single(ws[0])
    log(f"[bench] golden traces: {job.golden_s:.3f}s")

    # Plain fault-parallel kernel (K2).
    psteps = min(args.steps, PLAIN_STEPS)
    plain = None
    if args.only_headline:
        pass
    elif multi:
        plain = job.run_plain(psteps, min(args.warmup, 1))
    else:
        plain = job.run(riros.MODE_PLAIN, psteps, min(args.warmup, 1), {})
    if plain:
        log(f"[bench] plain: kernel {plain['kernel_ms']:.3f} ms, rate {rate(plain):.4g} FC/s")

    # Predictor: trained on held-out designs' plain-kernel events.
    pred_info, preds, wts, feats = {}, None, None, None
    if not args.no_predictor:
        wts, pred_info = train_predictor()
        t = time.perf_counter()
        feats = job.features()
        preds = [riros.mlp_predict(wts, f) for f in feats] if multi else riros.mlp_predict(wts, feats)
        pred_info["features_and_inference_s"] = time.perf_counter() - t
        if plain:
            true = np.concatenate([np.log2(1 + e.astype(np.float64)) for e in plain["events_arr"]])
            allf = np.concatenate(feats) if multi else feats
            err = predictor.load_error(np.concatenate(preds) if multi else preds, true)
            bsf, (bk, bsg) = best_single_feature(allf, true)
            pred_info.update({"spearman": err["spearman"], "mean_abs_log2": err["mean_abs_log2"],
                              "best_single_feature": {"index": int(bk), "sign": int(bsg), "spearman": bsf}})
            log(f"[bench] predictor: spearman {err['spearman']:.3f} (best single feature {bsf:.3f}), "
                f"mean |dlog2| {err['mean_abs_log2']:.3f}")

    # Autotuned two-dimensional schedule (bounded: a wall budget, and for long
    # lists a seeded sample of the faults).
    tuner = autotune.Autotuner(progress=log, budget_s=TUNE_BUDGET_S)
    t = time.perf_counter()
    if args.params:
        params = dict(autotune.DEFAULT, **json.loads(args.params))
    elif args.no_tune:
        params = dict(autotune.DEFAULT)
    elif multi:
        params = tuner.tune_batch([w.design for w in ws], job.ds, job.gs, [w.faults for w in ws], preds)
    else:
        F = ws[0].faults.size
        sample = None
        if F > TUNE_SAMPLE:
            sample = np.sort(np.argsort(W.counter_values(0x7E57, 0, F), kind="stable")[:TUNE_SAMPLE])
        params = tuner.tune_single(ws[0].design, job.d, job.g, ws[0].faults, preds, ws[0].T, sample=sample)
    tune_s = time.perf_counter() - t
    log(f"[bench] autotuner: {params} in {tune_s:.2f}s")

    # The ablation ladder: static order all light; a static heuristic (the
    # site's cone size) under the same heavy rule as the network, then with the
    # workgroup-wide heavy split; the network.
    ladder = {}
    static = None
    if multi:
        allp = None if preds is None else np.concatenate(preds)
        if not args.only_headline:
            static = job.run_batch(psteps, 1, autotune.batch_kwargs(dict(params, heavy_quantile=None)), None)
        best = job.run_batch(args.steps, args.warmup, autotune.batch_kwargs(params, allp), preds)
    else:
        if not args.only_headline:
            job.set_priority(None)
            static = job.run(riros.MODE_TWO_D, psteps, 1,
                             autotune.single_kwargs(dict(params, heavy_quantile=None)))
            if feats is not None:
                cone = np.ascontiguousarray(feats[:, 0], np.float32)
                job.set_priority(cone)
                heur = job.run(riros.MODE_TWO_D, psteps, 1, autotune.single_kwargs(params, cone))
                ladder["static_cone_heuristic"] = {"fault_cycles_per_s": rate(heur),
                                                   "kernel_ms": heur["kernel_ms"],
                                                   "identical": bool(same_results(heur, plain))}
                # The same static order with the workgroup-wide heavy split:
                # the top 1% by cone size start on four-wavefront structural
                # workgroups (the ladder's "+ heavy split" step).
                split = dict(params, heavy_quantile=0.99, heavy_wg=256, struct_share=4)
                hs = job.run(riros.MODE_TWO_D, psteps, 1, autotune.single_kwargs(split, cone))
                ladder["static_cone_heavy_wg_split"] = {"fault_cycles_per_s": rate(hs), "kernel_ms": hs["kernel_ms"],
                                                        "identical": bool(same_results(hs, plain))}
        job.set_priority(preds)
        best = job.run(riros.MODE_TWO_D, args.steps, args.warmup, autotune.single_kwargs(params, preds))
    if static:
        log(f"[bench] two_d static: kernel {static['kernel_ms']:.3f} ms")
    log(f"[bench] two_d with predictor: kernel {best['kernel_ms']:.3f} ms")
    same = (plain is None or same_results(plain, best)) and (static is None or same_results(static, best))

    # The paper keeps every fault for every cycle (no dropping): one extra run
    # in that convention on a seeded sample of the fault list, reported as
    # nominal F*T per second of kernel time.
    nodrop = None
    if args.no_drop_leg != "off" and not multi:
        w = ws[0]
        rank = np.argsort(W.counter_values(0xD0D0, 0, w.faults.size), kind="stable")

        def nd_run(sel, p, runs=2):
            pr_s = None if preds is None else np.ascontiguousarray(preds[sel], np.float32)
            kw = autotune.single_kwargs(p, pr_s)
            for _ in range(runs):   # the first run also loads code objects
                det_s, ev_s, _ = riros.fault_sim(job.d, job.g, np.ascontiguousarray(w.faults[sel]),
                                                 mode=riros.MODE_TWO_D, drop=False, priority=pr_s, **kw)
            return det_s, ev_s, riros.last_kernel_ms()

        # A design whose detected faults keep diverging across most of it
        # every cycle (no dropping) can take seconds per thousand faults: the
        # drop-mode schedule is timed on the sample's first faults, and when
        # the whole sample would take too long the leg keeps those (tuned
        # when a pass over them is short enough).
        probe = np.sort(rank[:min(w.faults.size, NO_DROP_PROBE)])
        _, _, probe_ms = nd_run(probe, params)
        n, tune_nd = no_drop_sample(w.faults.size, probe.size, probe_ms)
        tune_nd = tune_nd and not (args.params or args.no_tune)
        idx = np.sort(rank[:n])
        pr = None if preds is None else np.ascontiguousarray(preds[idx], np.float32)
        fl_nd = np.ascontiguousarray(w.faults[idx])
        # Without dropping, a detected fault keeps diverging for every
        # remaining cycle, so more of them outgrow a lane and run whole on the
        # structural path: the lane capacity, the monitor, the unified
        # schedule and the structural workgroup size are tuned again for this
        # convention, from the drop-mode point (the rest of the schedule is
        # kept).
        t = time.perf_counter()
        if tune_nd:
            nd_tuner = autotune.Autotuner(progress=log, budget_s=NO_DROP_TUNE_BUDGET_S)
            nd_params = nd_tuner.tune_single(w.design, job.d, job.g, fl_nd, pr, w.T, drop=False, start=params,
                                             names=NO_DROP_TUNED)
        else:
            nd_params = params
        nd_tune_s = time.perf_counter() - t
        ndet, nev, nd_ms = nd_run(idx, nd_params)
        FT = n * w.T
        nodrop = {"sample_faults": n, "nominal_fault_cycles_per_s": FT / (nd_ms * 1e-3), "fault_cycles": FT,
                  "kernel_ms": nd_ms, "events": int(nev.sum()),
                  "detect_identical": bool(np.array_equal(ndet, best["detect"][0][idx])),
                  "params": nd_params, "tune_s": nd_tune_s,
                  "probe": {"faults": int(probe.size), "kernel_ms": probe_ms}}
        log(f"[bench] no-drop sample of {n}: kernel {nd_ms:.3f} ms, {nodrop['nominal_fault_cycles_per_s']:.4g} F*T/s, "
            f"params {nd_params} (tuned in {nd_tune_s:.1f}s)")

    # The node-major alternative (faults grouped by site, 64 to a wavefront,
    # over the union of their frontiers) on the same inputs: at most two timed
    # steps, since it can be several times slower.
    conc = None
    if args.concurrent_leg != "off" and not multi:
        cr = job.run(riros.MODE_CONCURRENT, psteps, 1, {})
        conc = {"fault_cycles_per_s": rate(cr), "kernel_ms": cr["kernel_ms"], "steps": psteps,
                "identical_to_two_d": bool(same_results(cr, best))}
        same = same and conc["identical_to_two_d"]
        log(f"[bench] concurrent: kernel {cr['kernel_ms']:.3f} ms, rate {conc['fault_cycles_per_s']:.4g} FC/s")

    # Measured peaks (the published ones are the roofline's peaks).
    hbm_meas = riros.peak_hbm_gbs(2 << 30, 5)
    valu_meas = riros.peak_valu_ops(5)
    log(f"[bench] measured peaks: HBM stream {hbm_meas:.0f} GB/s, int32 VALU {valu_meas:.4g} op/s")

    FC, E, WD = best["fault_cycles"], best["events"], best["words"]
    value = rate(best)
    alg_bytes = BYTES_PER_WORD * WD
    achieved = alg_bytes / (best["kernel_ms"] * 1e-3) / 1e9
    ops_alg = OPS_PER_EVENT * E + OPS_PER_FC * FC
    ops_rate = ops_alg / (best["kernel_ms"] * 1e-3)
    total_faults = sum(w.faults.size for w in ws)
    ladder = {"plain": None if plain is None else {"fault_cycles_per_s": rate(plain), "kernel_ms": plain["kernel_ms"]},
              "two_d_static_all_light": None if static is None else
              {"fault_cycles_per_s": rate(static), "kernel_ms": static["kernel_ms"]},
              **ladder,
              "two_d_predictor": {"fault_cycles_per_s": value, "kernel_ms": best["kernel_ms"]}}
    out = {
        "metric": "fault-cycles/sec, plain vs batched+predictor, bit-exact detect cycles",
        "value": value, "unit": "fault-cycles/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": best["wall_s"] / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "designs": len(ws), "faults": int(total_faults),
                   "mode": "two-dimensional, predictor-ordered, autotuned" + (", one graph launch" if multi else "")},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(args.workload),
                     "kernel": "k_twod_a+k_twod_b", "kernel_ms": best["kernel_ms"],
                     "alg_bytes_per_launch": alg_bytes, "words": WD, "events": E, "fault_cycles": FC,
                     "measured_peak": hbm_meas, "frac_of_measured_peak": achieved / hbm_meas},
        "valu": {"ops_alg": ops_alg, "achieved": ops_rate, "peak": VALU_PEAK_OPS, "unit": "int32 op/s",
                 "frac": ops_rate / VALU_PEAK_OPS, "measured_peak": valu_meas,
                 "frac_of_measured_peak": ops_rate / valu_meas},
        "host": host_info(),
        "ablation": ladder,
        "plain": ladder["plain"],
        "two_d_predictor": ladder["two_d_predictor"],
        "speedup_vs_plain": None if plain is None else value / rate(plain),
        "autotuned": {"params": params, "tune_s": tune_s, "budget_s": TUNE_BUDGET_S,
                      "sample_faults": min(total_faults, TUNE_SAMPLE) if not multi else total_faults,
                      "whole_list_params": list(autotune.SCALE_PARAMS)
                      if not multi and total_faults > TUNE_SAMPLE else []},
        "predictor": pred_info,
        "no_drop": nodrop,
        "concurrent": conc,
        "golden_s": job.golden_s, "fault_cycles": FC, "events": E, "words": WD, "detected": best["detected"],
    }
    if args.campaign_leg != "off" and not multi:
        del job.f_dev
        torch.cuda.empty_cache()
        out["campaign"] = camp = campaign_leg(args, wts)
        same = same and camp["results_identical"]
    out["results_identical_across_modes"] = bool(same)

    if not args.no_cpu_baseline:
        import oracle
        nt = oracle.default_threads()
        # Parity over every fault of the (first) design and the CPU baseline:
        # the oracle's O1 on the whole list, timed on all host threads (its
        # golden trace, like the GPU's, is set-up and not timed).
        w = ws[0]
        t = time.perf_counter()
        G = oracle.golden(w.design, w.stimulus, w.T)
        g_s = time.perf_counter() - t
        log(f"[bench] oracle golden trace: {g_s:.1f}s")
        t = time.perf_counter()
        odet, oev, owk, _ = oracle.fault_sim_stats(w.design, w.stimulus, w.T, w.faults, G=G, nthreads=nt)
        cpu_s = time.perf_counter() - t
        cpu_fc = oracle.fault_cycles(odet, w.T)
        exact = bool(np.array_equal(odet, best["detect"][0]) and np.array_equal(oev, best["events_arr"][0]))
        if not multi:
            exact = exact and bool(np.array_equal(owk, best["words_arr"][0]))
        log(f"[bench] oracle O1 on all {w.faults.size} faults: {cpu_s:.1f}s, parity {'ok' if exact else 'MISMATCH'}")
        out["cpu_baseline"] = {"value": cpu_fc / cpu_s, "unit": "fault-cycles/s", "cores": nt, "kind": "oracle",
                               "sample": f"all {w.faults.size} faults of {w.name} (every fault compared with the GPU "
                                         f"run, detect, events and words), oracle O1 (divergent nodes only), "
                                         f"{cpu_s:.2f}s wall on {nt} threads; its golden trace ({g_s:.1f}s) untimed"}
        # One host thread on the first faults of a seeded draw (the paper
        # compares 1 and 16 cores), about 3 s.
        perm = np.argsort(W.counter_values(0xBA5E, 0, w.faults.size))
        fc1, s1, n1, n = 0, 0.0, 0, min(w.faults.size, 100)
        while n1 < w.faults.size and s1 < 3.0:
            idx = np.sort(perm[n1:n1 + n])
            t = time.perf_counter()
            odet1, _ = oracle.fault_sim(w.design, w.stimulus, w.T, w.faults[idx], G=G, variant=1, nthreads=1)
            s1 += time.perf_counter() - t
            fc1 += oracle.fault_cycles(odet1, w.T)
            n1 += idx.size
            exact &= bool(np.array_equal(odet1, odet[idx]))
            n = min(w.faults.size - n1, 2 * n)
        del G
        out["cpu_1thread"] = {"value": fc1 / s1, "unit": "fault-cycles/s", "cores": 1, "kind": "oracle",
                              "sample": f"{n1} faults of the same list (seeded draw), {s1:.2f}s on one thread"}
        out["parity"] = "bit-exact over every fault" if exact else "MISMATCH"
        if not exact:
            log("[bench] detect/events/words differ from the oracle")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
