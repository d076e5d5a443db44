"""Host-side parts of bench.py's contract (not gpu): the one-GPU guard and the rule that a
counter summary only counts for the kernel source it was taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_traffic_summary_is_dropped_when_the_kernel_source_changes(monkeypatch):
    for workload in ("cavity32", "es64"):
        for phase, hasher in (("spmv", "spmv_source_hash"), ("condense", "assembly_source_hash")):
            with open(os.path.join(ROOT, "profiles", f"{workload}_{phase}_traffic.json")) as f:
                stored = json.load(f)
            monkeypatch.setattr(bench, hasher, lambda: stored["source_sha256"])
            traffic, src = bench.measured_traffic(workload, phase)
            assert traffic == stored["traffic_bytes_per_launch"] and "stale" not in src
            monkeypatch.setattr(bench, hasher, lambda: "0" * 64)
            traffic, src = bench.measured_traffic(workload, phase)
            assert traffic is None and "stale" in src
    assert bench.measured_traffic("cavity32", "dots") == (None, None)     # no summary for that phase
