"""The benchmark script's host-side contract (no GPU needed): one GPU only, every
workload with its oracle sample, and the multipole kick's operation count."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], stdout=subprocess.PIPE,
                       stderr=subprocess.PIPE, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_every_workload_has_an_oracle_sample():
    assert set(bench.WORKLOADS) == set(bench.DEFAULT_CPU_STEPS)
    assert all(n > 0 for n in bench.DEFAULT_CPU_STEPS.values())


def test_multipole_operation_count():
    """45 (l, m >= 0) terms of 60 operations, 5 per degree and 60 per particle at
    lmax = 8 (the count the second kick's roofline uses)."""
    assert bench.mp_flops_per_particle(8) == 45 * 60 + 9 * 5 + 60 == 2805


def test_traffic_only_for_matching_sources(monkeypatch):
    """The measured traffic is read only when the counters were taken on the
    current kernel sources (and only at the 2^20 size they were taken at)."""
    assert bench.measured_traffic(1 << 22) is None
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
    assert bench.measured_traffic(1 << 20) is None
