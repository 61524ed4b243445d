"""The benchmark's host-side contract (no GPU): it refuses more than one GPU
with a message, and the committed HBM-traffic summaries it folds into the
roofline still describe the kernels as they stand in the source (a summary
goes stale, and the roofline's traffic field null, when a kernel's source
region changes)."""
import os
import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused(root):
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_summaries_match_the_kernel_sources():
    for kernel in bench.KERNELS:
        t = bench.read_traffic(kernel)
        assert t is not None and t > 0, kernel
