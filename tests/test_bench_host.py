"""Host-side logic of bench.py: the pair count behind the algorithmic work, the
traffic key, and the one-GPU guard (no GPU needed)."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("H,W,R", [(1, 1, 2), (5, 7, 2), (12, 9, 5), (4, 30, 3), (16, 16, 15)])
def test_window_pairs_counts_ordered_in_image_pairs(H, W, R):
    n = 0
    for y in range(H):
        for x in range(W):
            for a in range(-R, R + 1):
                for b in range(-R, R + 1):
                    if (a or b) and 0 <= y + a < H and 0 <= x + b < W:
                        n += 1
    assert bench.window_pairs(H, W, R) == n


def test_flops_per_pair_at_three_channels():
    assert bench.flops_per_pair(3, "fwd") == 23 and bench.flops_per_pair(3, "adj") == 54


def test_traffic_is_reported_only_for_the_profiled_kernel_source():
    assert bench.profiled_traffic("adj_step_kernel<3,5>") in (None, bench.PROFILED_TRAFFIC["adj_step_kernel<3,5>"])
    if bench.PROFILED_TRAFFIC["kernel_sha256"] == bench.kernel_sha():
        assert bench.profiled_traffic("adj_step_kernel<3,5>") > 0
    assert bench.profiled_traffic("no_such_kernel") is None


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
