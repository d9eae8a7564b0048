"""The benchmark's command-line contract, on the CPU (no GPU is touched):
more than one GPU is refused with a message, and the stored HBM counter
summary was taken on the fused kernels as they are (their source hash)."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "4"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr and "--gpus 4" in r.stderr
    assert r.stdout == ""


def test_counter_summary_matches_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    with open(bench.PMC_SUMMARY) as f:
        pm = json.load(f)
    assert pm["kernel_sha256_16"] == bench.kernel_hash()
    assert pm["hbm_bytes_per_launch"] > 0

