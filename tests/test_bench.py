"""CPU checks of bench.py's contract pieces that need no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


def test_algorithmic_counts_of_the_headline_workload():
    import bench

    # the method's algorithmic count on its reduced forms (P = M(M+1)/2 pairs):
    # 40 + 57 K + 10 M + 6 K M + 20 K M + 8 K P + P at 3 detectors, 21 modes
    assert bench.survey_flops_per_sample(3, 21) == 7834
    assert bench.survey_flops_per_sample(2, 2) == 40 + 114 + 20 + 24 + 80 + 48 + 3
    # the build's own formulation (harmonic-basis contraction), reported beside it
    assert bench.flops_per_sample(3, 21, 4) == 5012
    # theta (7 doubles) in, lnL out
    assert bench.bytes_per_sample() == 64


def test_traffic_is_keyed_to_the_kernel_sources():
    import bench

    t = bench.bench_traffic()
    # either the committed summary matches the current device code, or it is
    # reported as unknown: never a stale number
    assert t is None or t > 64e6
