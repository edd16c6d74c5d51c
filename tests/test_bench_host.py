"""Host-side checks of bench.py: the one-GPU contract and the algorithmic
counts its roofline uses (no GPU work)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_fine_flops_per_point_step_is_four_n():
    # one linear fine step = 4 folded sine-transform stages of 2 (n/2)^2 n
    # multiply-adds over n^2 points: 4 n flops per point (the unfolded count is 8 n)
    sys.path.insert(0, ROOT)
    import bench
    for n in (32, 64, 128, 256):
        stages = 4 * 2 * (n // 2) ** 2 * n * 2   # flops of the four folded stages
        assert bench.fine_flops_per_point_step(n) == stages / (n * n)


def test_traffic_constants_are_counter_based_and_positive():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.FINE_LAUNCH_TRAFFIC_BYTES is None or bench.FINE_LAUNCH_TRAFFIC_BYTES > 1e9
    assert (bench.PIPE_TRAFFIC_BYTES_PER_ITERATION is None
            or bench.PIPE_TRAFFIC_BYTES_PER_ITERATION > 1e9)
