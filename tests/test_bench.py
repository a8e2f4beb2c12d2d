"""Host-side contract of bench.py: the one-GPU exit, the committed traffic summary it reads, and the
full-size oracle comparison it makes only for the workload the stored result belongs to."""
import json
import os
import subprocess
import sys

import numpy as np

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    msg = json.loads(lines[0])
    assert "one GPU" in msg["error"] and msg["n_gpus"] == 2


def test_traffic_summary_matches_the_reduction_source():
    # the counter-measured bytes are reported only while the kernels they were taken on are unchanged
    tb = bench.traffic_bytes_per_launch()
    assert tb is not None, "profiles/gram_schmidt_traffic.txt was not taken on the current k_krylov.hip"
    vals = dict(ln.split(":", 1) for ln in open(bench.TRAFFIC) if ":" in ln)
    alg = float(vals["algorithmic_bytes_per_launch_avg"])
    # within a few percent of the algorithmic bytes: padding rows plus cache effects, no wasted re-reads
    assert 0.95 < tb / alg < 1.10


def test_oracle_comparison_only_for_its_workload():
    n = 1023 ** 2
    u = np.zeros(n)
    assert bench.golden_error(u, 20, "radau3", workload_matches=False) is None
    assert bench.golden_error(u, 20, "gl4") is None
    assert bench.golden_error(np.zeros(10), 20, "radau3") is None
