"""Benchmark of the fused fugacity-LBM step on one MI355X.

Workload: ten-component n-alkane mixture (C1..C10, seeded k_ij in [0, 0.05)),
D2Q9 1024 x 1024, spinodal start (uniform lever-rule density +-1 % seeded
noise), BGK tau = 1.  One step = moments, PR fugacity, interface potential,
force, collision and streaming of every population (one fused launch), plus
the mass / momentum / residual diagnostics every 100 steps.

Prints ONE JSON line.  ``value`` is component-site updates per second with
FP64 populations; the FP32-storage variant (FP64 arithmetic) is reported
alongside.  The dominant kernel's duration comes from HIP events recorded on
the stream the library launches on; HBM traffic per launch comes from the
committed rocprofv3 counter summary when it was taken on the current kernel
source.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "spinodal10_d2q9_1024x1024"
PMC_SUMMARY = os.path.join(ROOT, "profiles", "fused_d2q9_spinodal10_1024_pmc.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2306_10652_amd", "csrc", "kernels_fused2d.hip")


def kernel_hash():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def build_inputs(n):
    from inputs import components as C
    from inputs import fields as Fi
    st = Fi.load_phase_states()["spinodal10"]
    rho = Fi.add_noise(Fi.uniform(n, n, st["rho_uniform"]), 1e-2, 4)
    return C.N_ALKANES, 325.0, np.array(st["kij"]), rho


def time_gpu(precision, steps, warmup, n, diag_every=100):
    import torch
    from paper_2306_10652_amd import capi
    comps, T, kij, rho = build_inputs(n)
    mix = capi.Mixture.from_components(comps, T, kij, kappa_ref=0.02, tau=1.0)
    stream = torch.cuda.Stream()
    sim = capi.Simulation(mix, capi.D2Q9, precision, (n, n), rho, stream=stream)
    info = sim.info()
    sim.step_n(warmup)
    sim.diagnostics()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    # pure kernel time: HIP events on the library's stream around the steps
    kern_ms = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    d = None
    while done < steps:
        k = min(diag_every, steps - done)
        ev0.record(stream)
        sim.step_n(k)
        ev1.record(stream)
        d = sim.diagnostics()           # synchronises the stream
        kern_ms += ev0.elapsed_time(ev1)
        done += k
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    N = mix.N
    csu = N * n * n * steps / wall
    launch_s = kern_ms * 1e-3 / steps
    alg = info["alg_bytes_per_step"]
    res = dict(csu=csu, wall=wall, ms_per_step=wall * 1e3 / steps, launch_ms=launch_s * 1e3,
               alg_bytes=alg, achieved_gbs=alg / launch_s / 1e9, kernel=info["kernel"],
               status=d["status"], residual=d["residual"], mass=d["mass"].tolist())
    sim.close()
    return res


def cpu_baseline(n, budget_s=15.0):
    """The CPU oracle on a bounded sample: whole 1024^2 steps until ~budget."""
    from oracle.lbm import OracleLBM, oracle_mixture, build_oracle
    build_oracle()
    comps, T, kij, rho = build_inputs(n)
    m = oracle_mixture(comps, T, kij, kappa_ref=0.02, tau=1.0)
    o = OracleLBM(m, 0, (n, n), rho)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    k = 0
    while True:
        o.run(1)
        k += 1
        if time.perf_counter() - t0 > budget_s or k >= 20:
            break
    dt = time.perf_counter() - t0
    return dict(value=len(comps) * n * n * k / dt, unit="CSU/s", cores=threads, kind="oracle",
                sample="%d full step(s) of the %dx%d ten-component field (FP64, OpenMP), %.1f s"
                       % (k, n, n, dt))


def pmc_traffic(launch_alg_bytes):
    if not os.path.exists(PMC_SUMMARY):
        return None
    with open(PMC_SUMMARY) as f:
        pm = json.load(f)
    if pm.get("kernel_sha256_16") != kernel_hash():
        return None
    return pm.get("hbm_bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--precision", choices=["both", "fp64", "fp32"], default="both",
                    help="restrict the GPU legs (profiling runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB, 5 times "
                         "(calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.calib_copy_mib:
        import torch
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(calib_copy_bytes=n * 4, launches=5)))
        return
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; --gpus %d is not supported "
              "(multi-GPU sharding is design-only)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.precision != "both":
        r = time_gpu(0 if args.precision == "fp64" else 1, args.steps, args.warmup, args.n)
        print(json.dumps(dict(precision=args.precision, **{k: v for k, v in r.items()
                                                             if k != "mass"})), flush=True)
        return
    r64 = time_gpu(0, args.steps, args.warmup, args.n)
    r32 = time_gpu(1, args.steps, args.warmup, args.n)
    traffic = pmc_traffic(r64["alg_bytes"])
    roof = dict(bound="hbm", achieved=round(r64["achieved_gbs"], 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(r64["achieved_gbs"] / HBM_PEAK_GBS, 4),
                traffic=traffic, alg_bytes_per_launch=r64["alg_bytes"],
                launch_ms=round(r64["launch_ms"], 5), kernel="k_fused_d2q9<10,double>")
    out = dict(metric="component-site updates/s & %HBM roofline", value=round(r64["csu"], 1),
               unit="CSU/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=round(r64["ms_per_step"], 5), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f64", data="synthetic",
               config=dict(workload=WORKLOAD, grid=[args.n, args.n], components=10,
                           lattice="D2Q9", storage="fp64", tau=1.0, diag_every=100),
               roofline=roof,
               fp32_storage=dict(value=round(r32["csu"], 1), unit="CSU/s",
                                 ms_per_step=round(r32["ms_per_step"], 5),
                                 achieved_gbs=round(r32["achieved_gbs"], 1),
                                 frac=round(r32["achieved_gbs"] / HBM_PEAK_GBS, 4),
                                 alg_bytes_per_launch=r32["alg_bytes"],
                                 launch_ms=round(r32["launch_ms"], 5)),
               status=[r64["status"], r32["status"]])
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.n, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
