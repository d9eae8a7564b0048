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
KERNEL_SRCS = [os.path.join(ROOT, "paper_2306_10652_amd", "csrc", f)
               for f in ("lbm_common.h", "fused_common.h", "kernels_fused2d.hip",
                         "kernels_fused2d_ws.hip")]
KERNEL_NAMES = {2: "k_fused_d2q9<10,%s>", 3: "k_fused_d2q9_ws<10,%s>"}


def kernel_name(kernel, st):
    """Name of the step kernel the library ran (storage type st)."""
    return KERNEL_NAMES[kernel] % st if kernel in KERNEL_NAMES else "multi-pass (generic)"


def kernel_hash():
    """Hash of the fused kernels' sources (the profile summary records the
    hash it was measured with; a changed kernel voids its traffic figure)."""
    h = hashlib.sha256()
    for p in KERNEL_SRCS:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def build_inputs(n):
    from inputs import components as C
    from inputs import fields as Fi
    st = Fi.load_phase_states()["spinodal10"]
    rho = Fi.add_noise(Fi.uniform(n, n, st["rho_uniform"]), 1e-2, 4)
    return C.N_ALKANES, 325.0, np.array(st["kij"]), rho


def time_gpu(precision, steps, warmup, n, diag_every=100, rows=0, kernel=0, steady_steps=0):
    import torch
    from paper_2306_10652_amd import capi
    comps, T, kij, rho = build_inputs(n)
    mix = capi.Mixture.from_components(comps, T, kij, kappa_ref=0.02, tau=1.0)
    stream = torch.cuda.Stream()
    sim = capi.Simulation(mix, capi.D2Q9, precision, (n, n), rho, stream=stream)
    if rows or kernel:
        sim.set_tuning(kernel, rows)    # fixed rows: no tuning launches (profiling runs)
    info = sim.info()
    sim.step_n(warmup)                  # the first call autotunes rows (not timed)
    tuning = sim.get_tuning()
    mass0 = np.array(sim.diagnostics()["mass"], dtype=float)
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
    res = dict(csu=csu, csu_per_step=N * n * n, wall=wall, ms_per_step=wall * 1e3 / steps,
               launch_ms=launch_s * 1e3, alg_bytes=alg, achieved_gbs=alg / launch_s / 1e9, kernel=tuning["kernel"],
               rows=tuning["rows"],
               status=d["status"], residual=d["residual"], mass=d["mass"].tolist(),
               mass_drift=float(np.max(np.abs(np.array(d["mass"], dtype=float) - mass0) / mass0)))
    if steady_steps:
        # after the timed window: a longer run on the same simulation, for
        # the rate once the GPU's clocks have settled under sustained load,
        # as five back-to-back repetitions (their mean and their median)
        reps = 5
        each = max(1, steady_steps // reps)
        per = []
        for _ in range(reps):
            ev0.record(stream)
            sim.step_n(each)
            ev1.record(stream)
            ev1.synchronize()
            per.append(ev0.elapsed_time(ev1) * 1e-3 / each)
        ls = float(np.mean(per))
        med = float(np.median(per))
        res["steady"] = dict(steps=each * reps, launch_ms=round(ls * 1e3, 5),
                             value=round(N * n * n / ls, 1), achieved_gbs=round(alg / ls / 1e9, 1),
                             frac=round(alg / ls / 1e9 / HBM_PEAK_GBS, 4),
                             median_of_5=dict(steps_each=each, launch_ms=round(med * 1e3, 5),
                                              value=round(N * n * n / med, 1),
                                              frac=round(alg / med / 1e9 / HBM_PEAK_GBS, 4)))
    sim.close()
    return res


def copy_rate(mib=1024, reps=10):
    """A plain device-to-device copy of `mib` MiB on this GPU (torch's copy,
    hipMemcpyAsync underneath), GB/s counting the bytes read and written:
    the machine's own read-plus-write reference beside the 8 TB/s peak."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) * 1e-3
    del a, b
    return 2.0 * n * 8 * reps / t / 1e9


def sweep_leg(steps=512, acc_steps=200000, acc_count=8):
    """Batched ternary sweep (256 C1/C3/nC10 instances, FP32 storage, one
    launch per step, graph-replayed) against the same instances stepped one
    after another in plain FP64.  Accuracy of FP32 storage at equilibrium:
    thin slabs (64 x 4) of the first acc_count instances run acc_steps in
    both precisions, bulk phases compared."""
    import torch
    from paper_2306_10652_amd import batch, capi
    from inputs import fields as Fi
    S = Fi.load_phase_states()["ternary_sweep"]
    specs = batch.ternary_specs(S)
    st = torch.cuda.Stream()
    a = batch.Sweep(specs, capi.FP32_STORAGE, stream=st)
    a.step(64)                          # includes the batch's rows autotuning
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.step(steps)
    torch.cuda.synchronize()
    ta = time.perf_counter() - t0
    csu = a.csu_per_step
    a.close()
    b = batch.Sweep(specs, capi.FP64, stream=st)
    b.step_sequential(8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step_sequential(steps // 4)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    b.close()
    # accuracy at equilibrium on thin slabs of the first instances
    sub = []
    for sp, inst in zip(specs[:acc_count], S["instances"]):
        sp = dict(sp)
        sp["shape"] = (64, 4)
        sp["rho"] = Fi.slab(64, 4, inst["rho_V"], inst["rho_L"], 0.5)
        sub.append(sp)
    a = batch.Sweep(sub, capi.FP32_STORAGE, stream=st)
    b = batch.Sweep(sub, capi.FP64, stream=st)
    a.step(acc_steps)
    b.step(acc_steps)
    er, ex = 0.0, 0.0
    for pa, pb in zip(a.phases(), b.phases()):
        er = max(er, abs(pa["rho_V"] / pb["rho_V"] - 1), abs(pa["rho_L"] / pb["rho_L"] - 1))
        ex = max(ex, float(np.max(np.abs(pa["x"] - pb["x"]))), float(np.max(np.abs(pa["y"] - pb["y"]))))
    a.close()
    b.close()
    v_a = csu * steps / ta
    v_b = csu * (steps // 4) / tb
    return dict(instances=len(specs), csu_per_step=csu,
                fp32_batched=dict(value=round(v_a, 1), unit="CSU/s", ms_per_step=round(ta / steps * 1e3, 4)),
                fp64_sequential=dict(value=round(v_b, 1), unit="CSU/s",
                                     ms_per_step=round(tb / (steps // 4) * 1e3, 4)),
                factor=round(v_a / v_b, 2),
                fp32_vs_fp64_equilibrium=dict(instances=acc_count, grid=[64, 4], steps=acc_steps,
                                              max_rel_phase_density=er,
                                              max_abs_mole_fraction=ex))


def _linear_fit(x, y):
    A = np.vstack([x, np.ones(len(x))]).T
    coef, *_ = np.linalg.lstsq(A, np.array(y), rcond=None)
    fit = A @ coef
    y = np.array(y)
    return coef, 1 - np.sum((y - fit) ** 2) / np.sum((y - np.mean(y)) ** 2)


def time_vs_n_leg(steps=2000, big=1024, big_steps=200):
    """Per-step time against component count: Table II cases 1-6 as
    256 x 32 flat slabs, FP64 (the paper reports linear growth in N), and
    the same with FP32 storage (wall time over `steps` steps).  These grids
    sit in the caches and the step is bound by latency, which grows with
    the wavefronts per SIMD of the fused kernel's N + 2 wavefronts rather
    than with N itself; the same slabs at big x big, where the step streams
    its populations from HBM, are timed too (HIP events over `big_steps`)."""
    import torch
    from paper_2306_10652_amd import capi
    from inputs import components as C
    from inputs import fields as Fi
    S = Fi.load_phase_states()
    Ns, us, us32, usb, usb32 = [], [], [], [], []
    st = torch.cuda.Stream()
    for case in range(1, 7):
        comps, T, _ = C.table_ii_components(case)
        v = S["vle%d" % case]
        rho = Fi.slab(256, 32, v["rho_V"], v["rho_L"], 0.5)
        mix = capi.Mixture.from_components(comps, T)
        for prec, out in ((capi.FP64, us), (capi.FP32_STORAGE, us32)):
            sim = capi.Simulation(mix, capi.D2Q9, prec, (256, 32), rho, stream=st)
            sim.step_n(256)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sim.step_n(steps)
            torch.cuda.synchronize()
            out.append((time.perf_counter() - t0) / steps * 1e6)
            sim.close()
        rho = Fi.slab(big, big, v["rho_V"], v["rho_L"], 0.5)
        for prec, out in ((capi.FP64, usb), (capi.FP32_STORAGE, usb32)):
            sim = capi.Simulation(mix, capi.D2Q9, prec, (big, big), rho, stream=st)
            sim.step_n(64)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            sim.step_n(big_steps)
            e1.record(st)
            e1.synchronize()
            out.append(e0.elapsed_time(e1) / big_steps * 1e3)
            sim.close()
        Ns.append(len(comps))
    coef, r2 = _linear_fit(Ns, us)
    coefb, r2b = _linear_fit(Ns, usb)
    coefb32, r2b32 = _linear_fit(Ns, usb32)
    return dict(grid=[256, 32], N=Ns, us_per_step=[round(u, 2) for u in us],
                slope_us_per_component=round(coef[0], 3), r2=round(float(r2), 4),
                us_per_step_fp32_storage=[round(u, 2) for u in us32],
                hbm_bound=dict(grid=[big, big], steps=big_steps,
                               us_per_step=[round(u, 2) for u in usb],
                               slope_us_per_component=round(coefb[0], 3), r2=round(float(r2b), 4),
                               us_per_step_fp32_storage=[round(u, 2) for u in usb32],
                               r2_fp32_storage=round(float(r2b32), 4)))


def serving_leg(count=10, load=0.8, tol=1e-8, max_steps=200000, max_n2d=None, max_n3d=None,
                largest=("D2Q9",)):
    """Continuous batching over requests of the stored pool at their own
    sizes (2-10 components; D2Q9 64^2 ... 512^2, D3Q19 64^3 ... 128^3): the
    first `count` of the pool plus its first requests at the largest sizes
    of the lattices in `largest` (the default leg leaves out the 128^3
    D3Q19 request, whose ~9e4 steps take ~90 s alone), FP32 storage, each
    run to residual tol or the step cap.  A first,
    closed-loop pass (every request present at t = 0) measures each
    request's work and the server's capacity; the timed pass then offers
    `load` x that capacity with Poisson arrivals.  Time-to-equilibrium
    percentiles are over the requests that converged; capped requests are
    counted apart."""
    import torch
    from paper_2306_10652_amd import capi, serve
    from inputs import fields as Fi
    S = Fi.load_phase_states()["serving_pool"]

    def progress_fn(tag):
        last = [0.0]

        def progress(t, active, waiting, done):
            if t - last[0] >= 15.0:
                last[0] = t
                print("serving %s: %.0f s, %d active, %d waiting, %d done"
                      % (tag, t, active, waiting, done), file=sys.stderr, flush=True)
        return progress

    pool = S["requests"]
    extra = []
    for lat in largest:
        nmax = max(q["n"] for q in pool if q["lattice"] == lat)
        extra.append(next(k for k, q in enumerate(pool) if q["lattice"] == lat and q["n"] == nmax))
    idx = list(range(count)) + [k for k in extra if k >= count]
    closed = serve.pool_requests(S, 0, rate_hz=1e9, tol=tol, max_steps=max_steps,
                                 max_n2d=max_n2d, max_n3d=max_n3d, indices=idx)
    for r in closed:
        r.arrival = 0.0
    t0 = time.perf_counter()
    done0 = serve.Server(64 << 30, chunk=200).run(closed, progress=progress_fn("closed"))
    wall0 = time.perf_counter() - t0
    work = [r.csu() for r in done0 if r.status == 0]
    capacity = sum(work) / wall0
    mean_work = float(np.mean(work))
    rate = load * capacity / mean_work
    reqs = serve.pool_requests(S, 0, rate_hz=rate, tol=tol, max_steps=max_steps,
                               max_n2d=max_n2d, max_n3d=max_n3d, seed=55, indices=idx)
    srv = serve.Server(64 << 30, chunk=200)
    t0 = time.perf_counter()
    done = srv.run(reqs, progress=progress_fn("open"))
    wall = time.perf_counter() - t0
    st = serve.latency_stats(done)
    csu = sum(r.csu() for r in done if r.status == 0)
    sizes = sorted(set((("D2Q9" if r.lattice == capi.D2Q9 else "D3Q19"), r.shape[0]) for r in reqs))
    st.update(max_n2d=max(n for l, n in sizes if l == "D2Q9"),
              max_n3d=max([n for l, n in sizes if l == "D3Q19"] or [0]),
              d3q19_requests=sum(r.lattice != capi.D2Q9 for r in reqs),
              offered_load=load, arrival_rate_hz=round(rate, 4),
              closed_loop=dict(wall_s=round(wall0, 2), capacity_csu_s=round(capacity, 1),
                               mean_work_csu=round(mean_work, 1)),
              hbm_budget_gb=64, tol=tol, max_steps=max_steps, wall_s=round(wall, 3),
              throughput=dict(value=round(csu / wall, 1), unit="CSU/s"))
    return st


def d3q19_leg(n=128, steps=100, warmup=10):
    """The largest D3Q19 request of the serving stream: the ten-component
    spinodal mixture on a n^3 periodic grid (uniform, +-1 % noise), FP64
    and FP32 storage, multi-pass path.  Kernel time from HIP events on the
    library's stream; traffic per step both as the populations alone (the
    headline's definition) and with the fields the passes exchange
    (8N + 14 values per site)."""
    import torch
    from paper_2306_10652_amd import capi
    from inputs import components as C
    from inputs import fields as Fi
    st = Fi.load_phase_states()["spinodal10"]
    rho = Fi.add_noise(Fi.uniform(n, n, st["rho_uniform"], nz=n), 1e-2, 4)
    mix = capi.Mixture.from_components(C.N_ALKANES, 325.0, np.array(st["kij"]),
                                       kappa_ref=0.02, tau=1.0)
    N, ns = mix.N, n ** 3
    stream = torch.cuda.Stream()
    out = dict(grid=[n, n, n], components=N, lattice="D3Q19", steps=steps)
    for prec, name in ((capi.FP64, "fp64"), (capi.FP32_STORAGE, "fp32_storage")):
        sim = capi.Simulation(mix, capi.D3Q19, prec, (n, n, n), rho, stream=stream)
        sim.step_n(warmup)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step_n(steps)
        e1.record(stream)
        e1.synchronize()
        s = e0.elapsed_time(e1) * 1e-3 / steps
        pop = sim.info()["alg_bytes_per_step"]
        fields = (8 * N + 14) * 8 * ns
        out[name] = dict(ms_per_step=round(s * 1e3, 4), value=round(N * ns / s, 1), unit="CSU/s",
                         populations_gbs=round(pop / s / 1e9, 1),
                         populations_frac=round(pop / s / 1e9 / HBM_PEAK_GBS, 4),
                         with_fields_gbs=round((pop + fields) / s / 1e9, 1),
                         status=sim.diagnostics()["status"])
        sim.close()
    return out


def small_workloads_leg(droplet_steps=2000, slab_steps=20000, window=200, sweep_window=2):
    """The oracle (all OpenMP threads and one thread) beside the GPU on the
    smaller workloads:
    * the 64^2 C1/C3/nC5 droplet: its full 2000 steps on the GPU (FP64,
      cache-resident: reported as steps/s and CSU/s) and on the oracle,
      with all threads and with one;
    * the 256 x 32 Table II slabs, N = 1..6: the oracle over each case's
      full 20000 steps with all threads, and over a `window`-step sample
      per case on one thread (the GPU side is the time-vs-N leg);
    * the 256 ternary sweep instances: the oracle over `sweep_window`
      steps of every instance, one after another.
    Oracle rates are CSU/s over the stated samples."""
    import torch
    from paper_2306_10652_amd import capi
    from inputs import components as C
    from inputs import fields as Fi
    from oracle.lbm import OracleLBM, oracle_mixture, build_oracle, set_threads
    build_oracle()
    S = Fi.load_phase_states()
    threads = set_threads(0)
    out = dict(cores=threads, cpu_model=cpu_model())
    # the 64^2 droplet
    st = S["droplet3"]
    rho = Fi.add_noise(Fi.droplet(64, 64, st["rho_L"], st["rho_V"], 16.0), 1e-3, 1)
    mix = capi.Mixture.from_components(C.DROPLET_3, 250.0)
    stream = torch.cuda.Stream()
    sim = capi.Simulation(mix, capi.D2Q9, capi.FP64, (64, 64), rho, stream=stream)
    sim.step_n(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step_n(droplet_steps)
    torch.cuda.synchronize()
    g = time.perf_counter() - t0
    sim.close()
    csu1 = 3 * 64 * 64
    om = oracle_mixture(C.DROPLET_3, 250.0)
    rates = {}
    for nt in (threads, 1):
        set_threads(nt)
        o = OracleLBM(om, 0, (64, 64), rho)
        t0 = time.perf_counter()
        o.run(droplet_steps)
        rates[nt] = csu1 * droplet_steps / (time.perf_counter() - t0)
        print("small_workloads: oracle, droplet, %d steps on %d thread(s)" % (droplet_steps, nt),
              file=sys.stderr, flush=True)
    out["droplet64_c1c3nc5"] = dict(
        gpu=dict(steps=droplet_steps, steps_per_s=round(droplet_steps / g, 1),
                 csu_s=round(csu1 * droplet_steps / g, 1)),
        oracle=dict(sample="%d steps (the full run)" % droplet_steps,
                    csu_s_all_cores=round(rates[threads], 1),
                    csu_s_one_thread=round(rates[1], 1)))
    # the Table II slabs
    c2, c2_1, c2_wall = [], [], []
    for case in range(1, 7):
        comps, T, _ = C.table_ii_components(case)
        v = S["vle%d" % case]
        rho2 = Fi.slab(256, 32, v["rho_V"], v["rho_L"], 0.5)
        csu2 = len(comps) * 256 * 32
        set_threads(threads)
        o = OracleLBM(oracle_mixture(comps, T), 0, (256, 32), rho2)
        t0 = time.perf_counter()
        o.run(slab_steps)
        dt = time.perf_counter() - t0
        c2.append(round(csu2 * slab_steps / dt, 1))
        c2_wall.append(round(dt, 2))
        print("small_workloads: oracle, Table II case %d, %d steps in %.1f s"
              % (case, slab_steps, dt), file=sys.stderr, flush=True)
        set_threads(1)
        o = OracleLBM(oracle_mixture(comps, T), 0, (256, 32), rho2)
        t0 = time.perf_counter()
        o.run(window)
        c2_1.append(round(csu2 * window / (time.perf_counter() - t0), 1))
    set_threads(threads)
    out["table_ii_slabs_256x32"] = dict(
        N=[1, 2, 3, 4, 5, 6], oracle_csu_s_all_cores=c2, oracle_wall_s_all_cores=c2_wall,
        sample_all_cores="%d steps per case (the full run)" % slab_steps,
        oracle_csu_s_one_thread=c2_1, sample_one_thread="%d steps per case" % window)
    # the ternary sweep instances
    from paper_2306_10652_amd import batch
    specs = batch.ternary_specs(S["ternary_sweep"])
    csu = 0
    el = 0.0
    for sp in specs:
        o = OracleLBM(oracle_mixture(sp["comps"], sp["T"]), 0, sp["shape"], sp["rho"])
        t0 = time.perf_counter()
        o.run(sweep_window)
        el += time.perf_counter() - t0
        csu += 3 * sp["shape"][0] * sp["shape"][1] * sweep_window
        del o
    out["ternary_sweep_256"] = dict(instances=len(specs), oracle_csu_s_all_cores=round(csu / el, 1),
                                sample="%d steps of each instance" % sweep_window)
    set_threads(threads)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, budget_s=15.0, gpu_check=True):
    """The CPU oracle on a bounded sample: whole 1024^2 steps until ~budget
    with every thread OpenMP gets, then one step on one thread.  The
    sample's end state also checks the GPU (gpu_check): the same input
    stepped as many times by the library (FP64, its benchmark launch
    configuration), densities compared over the whole field."""
    from oracle.lbm import OracleLBM, oracle_mixture, build_oracle, set_threads
    build_oracle()
    comps, T, kij, rho = build_inputs(n)
    m = oracle_mixture(comps, T, kij, kappa_ref=0.02, tau=1.0)
    o = OracleLBM(m, 0, (n, n), rho)
    threads = set_threads(0)
    t0 = time.perf_counter()
    k = 0
    while True:
        o.run(1)
        k += 1
        if time.perf_counter() - t0 > budget_s or k >= 20:
            break
    dt = time.perf_counter() - t0
    parity = None
    if gpu_check:
        from paper_2306_10652_amd import capi
        mix = capi.Mixture.from_components(comps, T, kij, kappa_ref=0.02, tau=1.0)
        sim = capi.Simulation(mix, capi.D2Q9, capi.FP64, (n, n), rho)
        sim.step_n(k)
        g = sim.read_moments(velocity=False)["rho"]
        ref = o.rho()
        parity = dict(steps=k, rho_max_rel=float(np.max(np.abs(g - ref) / ref)),
                      kernel=kernel_name(sim.info()["kernel"], "double"))
        sim.close()
        mix.close()
    set_threads(1)
    t1 = time.perf_counter()
    o.run(1)
    dt1 = time.perf_counter() - t1
    set_threads(threads)
    csu = len(comps) * n * n
    return dict(value=csu * k / dt, unit="CSU/s", cores=threads, kind="oracle",
                sample="%d full step(s) of the %dx%d ten-component field (FP64, OpenMP), %.1f s"
                       % (k, n, n, dt),
                one_thread=dict(value=csu / dt1, unit="CSU/s",
                                sample="1 full step on 1 thread, %.1f s" % dt1),
                gpu_vs_oracle=parity,
                nproc=os.cpu_count(), cpu_model=cpu_model())


def pmc_traffic(launch_alg_bytes):
    if not os.path.exists(PMC_SUMMARY):
        return None
    with open(PMC_SUMMARY) as f:
        pm = json.load(f)
    if pm.get("kernel_sha256_16") != kernel_hash():
        return None
    return pm.get("hbm_bytes_per_launch")


def trace_summary(db_path, steps, steady=0):
    """Per-kernel durations from a rocprofv3 results database (kernel-trace
    run of this script): every dispatch, and the timed window of each
    kernel, i.e. its `steps` dispatches before the last `steady` ones (for
    the fused step kernels: after the autotuner's trial launches and the
    warm-up, before the steady-state run).  Prints a markdown table."""
    import sqlite3
    db = sqlite3.connect(db_path)
    rows = list(db.execute("select name, start, end from kernels order by start"))
    by = {}
    for name, t0, t1 in rows:
        by.setdefault(name, []).append((t1 - t0) / 1e3)
    print("| kernel | calls | avg us (all) | timed window: calls | avg us | min us | max us |"
          " steady: avg us |")
    print("|---|---|---|---|---|---|---|---|")
    for name, d in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        short = name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        if len(d) <= steady + steps:
            # not a step kernel of the timed loop (trial launches, read-outs)
            print("| `%s` | %d | %.1f | | | | | |" % (short, len(d), sum(d) / len(d)))
            continue
        win = d[len(d) - steady - steps:len(d) - steady]
        tail = d[len(d) - steady:] if steady else []
        print("| `%s` | %d | %.1f | %d | %.1f | %.1f | %.1f | %s |" % (
            short, len(d), sum(d) / len(d), len(win), sum(win) / len(win), min(win), max(win),
            "%.1f" % (sum(tail) / len(tail)) if tail else "-"))


def marker_summary(db_path):
    """The library's roctx ranges (one per C-ABI call that launches work)
    from a rocprofv3 --marker-trace results database: calls, total and mean
    host time per range name.  Prints a markdown table."""
    import sqlite3
    db = sqlite3.connect(db_path)
    agg = {}
    for start, end, ext in db.execute("select start, end, extdata from regions "
                                      "where category = 'MARKER_CORE_RANGE_API' order by start"):
        name = json.loads(ext or "{}").get("message", "?")
        agg.setdefault(name, []).append((end - start) / 1e6)
    print("| range | calls | total ms | mean ms | max ms |")
    print("|---|---|---|---|---|")
    for name, d in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        print("| `%s` | %d | %.2f | %.3f | %.3f |" % (name, len(d), sum(d), sum(d) / len(d), max(d)))


def sq_summary(db_paths, kernel="k_fused_d2q9_ws"):
    """Median per dispatch of every counter in the given rocprofv3 counter
    databases (separate passes of one workload) for the kernels whose name
    contains `kernel`, and the wavefront-cycle fractions derived from them.
    Prints a markdown table."""
    import sqlite3
    import statistics
    vals = {}
    for path in db_paths:
        db = sqlite3.connect(path)
        for name, counter, value in db.execute(
                "select kernel_name, counter_name, value from counters_collection"):
            if kernel in name:
                vals.setdefault(counter, []).append(value)
    med = {c: statistics.median(v) for c, v in vals.items()}
    print("| counter | median per dispatch |")
    print("|---|---|")
    for c in sorted(med):
        print("| %s | %.0f |" % (c, med[c]))
    wc = med.get("SQ_WAVE_CYCLES")
    if wc:
        for c in ("SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_SCA", "SQ_WAIT_ANY",
                  "SQ_WAIT_INST_ANY", "SQ_WAIT_INST_LDS"):
            if c in med:
                print("| %s / SQ_WAVE_CYCLES | %.3f |" % (c, med[c] / wc))


def _counter_values(db_path, counter):
    """(kernel name, value) of every dispatch in a rocprofv3 counter-collection
    database, in dispatch order."""
    import sqlite3
    db = sqlite3.connect(db_path)
    return [(n, v) for n, v in db.execute(
        "select kernel_name, value from counters_collection where counter_name = ? "
        "order by dispatch_id", (counter,))]


def pmc_summary(out_path, fetch64, write64, fetch32, write32, calib_fetch, calib_write, steps,
                copy_bytes=1 << 30):
    """The HBM traffic summary of the fused kernel (profiles/ JSON read by
    this script): FETCH_SIZE and WRITE_SIZE (KiB per dispatch, separate
    counter runs of `--precision P --rows 74`) averaged over the last
    `steps` dispatches of the fused kernel, each scaled by what the counter
    reads for a plain device copy of `copy_bytes` (`--calib-copy-mib`)."""
    def copy_kib(path, counter):
        vals = [v for n, v in _counter_values(path, counter) if "copyBuffer" in n]
        return max(vals)
    f_fac = copy_bytes / (copy_kib(calib_fetch, "FETCH_SIZE") * 1024.0)
    w_fac = copy_bytes / (copy_kib(calib_write, "WRITE_SIZE") * 1024.0)
    per = {}
    for prec, fpath, wpath, st in (("fp64", fetch64, write64, "double"),
                                   ("fp32", fetch32, write32, "float")):
        kern = KERNEL_NAMES[3] % st
        fv = [v for n, v in _counter_values(fpath, "FETCH_SIZE") if kern in n.replace(" ", "")][-steps:]
        wv = [v for n, v in _counter_values(wpath, "WRITE_SIZE") if kern in n.replace(" ", "")][-steps:]
        rd = float(np.mean(fv)) * 1024.0 * f_fac
        wr = float(np.mean(wv)) * 1024.0 * w_fac
        alg = 2 * 10 * 1024 * 1024 * (8 + 8 * (8 if st == "double" else 4))
        per[prec] = dict(kernel=kern, dispatches=len(fv), fetch_kib_raw=float(np.mean(fv)),
                         write_kib_raw=float(np.mean(wv)), hbm_read_bytes_per_launch=rd,
                         hbm_write_bytes_per_launch=wr, hbm_bytes_per_launch=rd + wr,
                         alg_bytes_per_launch=alg, traffic_over_alg=(rd + wr) / alg)
    out = dict(kernel_sha256_16=kernel_hash(), workload=WORKLOAD,
               calibration=dict(copy_bytes=copy_bytes, fetch_factor=f_fac, write_factor=w_fac),
               hbm_bytes_per_launch=per["fp64"]["hbm_bytes_per_launch"], per_precision=per)
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--steady-steps", type=int, default=400,
                    help="after the timed window, time this many more steps of the same "
                         "simulation in five equal repetitions (reported as steady_state, "
                         "with their median; 0: skip)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the sweep, time-vs-N and serving legs")
    ap.add_argument("--legs", default="sweep,time_vs_n,serving,d3q19",
                    help="comma-separated extra legs to run (sweep, time_vs_n, serving, "
                         "d3q19; serving_more, the serving stream over more requests, and "
                         "small_workloads, the oracle beside the GPU on the 64^2 droplet, the "
                         "Table II slabs and the sweep instances, "
                         "run only when named)")
    ap.add_argument("--precision", choices=["both", "fp64", "fp32"], default="both",
                    help="restrict the GPU legs (profiling runs)")
    ap.add_argument("--rows", type=int, default=0,
                    help="fix the fused kernel's rows per work item instead of "
                         "autotuning (profiling runs: no tuning launches)")
    ap.add_argument("--kernel", type=int, default=0, choices=[0, 1, 2, 3],
                    help="fix the step kernel (0 = autotuned; 2 / 3 = the two fused "
                         "variants; with --rows and 0, the default fused variant)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB, 5 times "
                         "(calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    ap.add_argument("--trace-summary", default=None,
                    help="only summarise a rocprofv3 results database of a kernel-trace run "
                         "of this script (per-kernel durations; the last --steps dispatches "
                         "of each kernel are the timed window)")
    ap.add_argument("--sq-summary", nargs="+", default=None,
                    help="print the fused kernel's SQ counters (median per dispatch) from "
                         "rocprofv3 counter databases and exit")
    ap.add_argument("--marker-summary", default=None,
                    help="print the library's roctx ranges from a rocprofv3 --marker-trace "
                         "results database and exit")
    ap.add_argument("--pmc-summary", nargs=7, default=None,
                    metavar=("OUT", "FETCH64", "WRITE64", "FETCH32", "WRITE32", "CALIB_FETCH",
                             "CALIB_WRITE"),
                    help="only write the HBM traffic summary OUT from rocprofv3 counter "
                         "databases (FETCH_SIZE / WRITE_SIZE runs of --precision fp64 and fp32, "
                         "and of --calib-copy-mib 1024); the last --steps dispatches are used")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, steps=args.steps)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary, args.steps, args.steady_steps)
        return
    if args.marker_summary:
        marker_summary(args.marker_summary)
        return
    if args.sq_summary:
        sq_summary(args.sq_summary)
        return
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
        print("bench.py measures one GPU; --gpus %d is not supported "
              "(multi-GPU sharding is design-only)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    if args.precision != "both":
        r = time_gpu(0 if args.precision == "fp64" else 1, args.steps, args.warmup, args.n,
                     rows=args.rows, kernel=args.kernel)
        print(json.dumps(dict(precision=args.precision, **{k: v for k, v in r.items()
                                                             if k != "mass"})), flush=True)
        return
    r64 = time_gpu(0, args.steps, args.warmup, args.n, rows=args.rows, kernel=args.kernel,
                   steady_steps=args.steady_steps)
    r32 = time_gpu(1, args.steps, args.warmup, args.n, rows=args.rows, kernel=args.kernel,
                   steady_steps=args.steady_steps)
    traffic = pmc_traffic(r64["alg_bytes"])
    roof = dict(bound="hbm", achieved=round(r64["achieved_gbs"], 1), peak=HBM_PEAK_GBS,
                unit="GB/s", frac=round(r64["achieved_gbs"] / HBM_PEAK_GBS, 4),
                traffic=traffic, alg_bytes_per_launch=r64["alg_bytes"],
                launch_ms=round(r64["launch_ms"], 5),
                kernel=kernel_name(r64["kernel"], "double"),
                rows_per_item=r64["rows"])
    if "steady" in r64:
        roof["steady_state"] = r64["steady"]
    copy_gbs = copy_rate()
    roof["copy_gbs"] = round(copy_gbs, 1)
    roof["frac_of_copy"] = round(r64["achieved_gbs"] / copy_gbs, 4)
    out = dict(metric="component-site updates/s & %HBM roofline; p50/p99 time-to-equilibrium",
               value=round(r64["csu"], 1),
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
                                 launch_ms=round(r32["launch_ms"], 5),
                                 frac_72B=round(72 * r32["csu_per_step"] / (r32["launch_ms"] * 1e-3)
                                                / 1e9 / HBM_PEAK_GBS, 4),
                                 frac_of_copy=round(r32["achieved_gbs"] / copy_gbs, 4),
                                 kernel=kernel_name(r32["kernel"], "float"),
                                 rows_per_item=r32["rows"], steady_state=r32.get("steady")),
               status=[r64["status"], r32["status"]],
               mass_drift=[r64["mass_drift"], r32["mass_drift"]])
    legs = set() if args.no_extra else set(args.legs.split(","))
    if "sweep" in legs:
        out["batched_sweep"] = sweep_leg()
    if "time_vs_n" in legs:
        out["time_vs_N"] = time_vs_n_leg()
    if "serving" in legs:
        out["serving"] = serving_leg()
    if "d3q19" in legs:
        out["d3q19"] = d3q19_leg()
    if "small_workloads" in legs:
        out["small_workloads"] = small_workloads_leg()
    if "serving_more" in legs:
        out["serving_more"] = serving_leg(count=20, largest=("D2Q9", "D3Q19"))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.n, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
