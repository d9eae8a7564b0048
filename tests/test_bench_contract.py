"""The benchmark's contract, on the CPU (no GPU is touched): more than one
GPU is refused with a message, the stored HBM counter summary was taken on
the fused kernels as they are (their source hash), and the oracle leg runs."""
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



def test_cpu_baseline_leg_on_a_small_field():
    """The oracle leg of the benchmark (whole steps with every OpenMP thread,
    then one step on one thread) on a 64^2 field of the same mixture: the
    fields the bench line reports are there and positive."""
    sys.path.insert(0, ROOT)
    import bench
    r = bench.cpu_baseline(64, budget_s=0.2)
    assert r["kind"] == "oracle" and r["unit"] == "CSU/s"
    assert r["value"] > 0 and r["one_thread"]["value"] > 0
    assert r["cores"] >= 1 and "64x64" in r["sample"]
