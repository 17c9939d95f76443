"""Host-side parts of the benchmark: the committed traffic counters are used
only for the kernel sources they were taken on, and more than one GPU is
refused with a message."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_counters_are_used_only_for_their_sources():
    got = bench.measured_traffic("large")
    text = open(os.path.join(ROOT, "profiles", "traffic_large.md")).read()
    if f"`{bench.kernel_source_digest()}`" in text:
        assert got is not None and got > 0
        assert f"`{int(got)}`" in text
    else:
        assert got is None


def test_traffic_is_null_for_other_sources(monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "0000000000000000")
    assert bench.measured_traffic("large") is None
    assert bench.measured_traffic("no_such_workload") is None


def test_host_info_fields():
    h = bench.host_info()
    assert set(h) == {"cpu_model", "logical_cpus", "usable_cpus"}
    assert h["usable_cpus"] >= 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_no_drop_sample_keeps_the_probe_when_the_full_sample_is_too_slow():
    # large: 2,000 faults in 127 ms -> 20,000 in about 1.3 s, tuned
    assert bench.no_drop_sample(1_000_000, 2000, 127.0) == (bench.NO_DROP_SAMPLE, True)
    # medium: 2,000 faults in 1,193 ms -> about 12 s: the probe, tuned
    assert bench.no_drop_sample(50_000, 2000, 1193.0) == (2000, True)
    # a probe pass of several seconds: the probe, untuned
    assert bench.no_drop_sample(50_000, 2000, 5000.0) == (2000, False)
    # a list shorter than the sample: the whole list
    assert bench.no_drop_sample(1500, 1500, 5.0) == (1500, True)
