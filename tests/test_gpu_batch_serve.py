"""Batched sweeps and the continuous-batching server (GPU).

* A batched step (one launch for many uneven simulations, hipGraph-replayed)
  gives bitwise the same populations as stepping each simulation alone.
* FP32 storage against FP64 on the same batch: bulk phase densities within
  1e-4 relative and mole fractions within 1e-3 absolute.
* The full-size batched sweep, sampled instances against the oracle.
* The server: every request's result is bitwise the same alone and in the
  mix and matches the oracle; the HBM budget is never exceeded; a request
  that goes non-finite fails alone while the others finish normally.
"""
import numpy as np
import pytest

from tests import workloads as W
from tests.test_gpu_parity import _capi, report

pytestmark = pytest.mark.gpu


def small_specs(count=8, max_n=96):
    from paper_2306_10652_amd import batch
    specs = batch.ternary_specs(W.states()["ternary_sweep"], count=count)
    out = []
    from inputs import fields as Fi
    inst = W.states()["ternary_sweep"]["instances"]
    for sp, st in zip(specs, inst):
        n = min(st["n"], max_n) - (7 if len(out) % 2 else 0)   # uneven, ragged grids
        sp = dict(sp)
        sp["shape"] = (n, n)
        sp["rho"] = Fi.slab(n, n, st["rho_V"], st["rho_L"], st["S_V"])
        out.append(sp)
    return out


def test_batched_equals_single_bitwise():
    capi = _capi()
    from paper_2306_10652_amd import batch
    specs = small_specs()
    sw = batch.Sweep(specs, capi.FP32_STORAGE)
    sw.step(75)       # long enough to autotune rows for this batch shape
    sw.step(125)      # graph-replayed runs + a remainder
    singles = batch.Sweep(specs, capi.FP32_STORAGE)
    singles.step_sequential(200)
    for a, b in zip(sw.sims, singles.sims):
        assert np.array_equal(a.read_populations(), b.read_populations())
    sw.close()
    singles.close()


def test_fp32_batch_against_fp64_equilibrium_phases():
    """FP32 storage against FP64 at equilibrium (thin ternary slabs run to a
    stationary state): bulk phase densities within 1e-4 relative and mole
    fractions within 1e-3 absolute (bulk = even-width window averages)."""
    capi = _capi()
    from paper_2306_10652_amd import batch
    from inputs import fields as Fi
    specs = []
    for sp, st in zip(batch.ternary_specs(W.states()["ternary_sweep"], count=6),
                      W.states()["ternary_sweep"]["instances"]):
        sp = dict(sp)
        sp["shape"] = (64, 4)
        sp["rho"] = Fi.slab(64, 4, st["rho_V"], st["rho_L"], 0.5)
        specs.append(sp)
    a = batch.Sweep(specs, capi.FP32_STORAGE)
    b = batch.Sweep(specs, capi.FP64)
    a.step(200000)
    b.step(200000)
    worst_rho, worst_x = 0.0, 0.0
    for pa, pb in zip(a.phases(), b.phases()):
        for ph in ("rho_V", "rho_L"):
            worst_rho = max(worst_rho, abs(pa[ph] / pb[ph] - 1))
        worst_x = max(worst_x, np.max(np.abs(pa["x"] - pb["x"])), np.max(np.abs(pa["y"] - pb["y"])))
    report("fp32_vs_fp64_equilibrium", rho_rel=worst_rho, x_abs=worst_x)
    assert worst_rho <= 1e-4 and worst_x <= 1e-3
    a.close()
    b.close()


def _bulk_by_gradient(sim, M, tol=1e-4):
    """Bulk phases of a flat slab by the gradient criterion: columns where
    max_i |grad rt_i| / rt_i < tol (central difference of the column means),
    split at the mid density into liquid and vapour; each phase's mean molar
    density and composition (None for a phase with no bulk column).  Does
    not depend on where the slab sits."""
    rt = sim.read_moments(velocity=False)["rho"][:, 0] / np.asarray(M)[:, None, None]
    p = rt.mean(axis=1)
    g = np.abs(np.roll(p, -1, axis=1) - np.roll(p, 1, axis=1)) / 2 / p
    ok = g.max(axis=0) < tol
    t = p.sum(axis=0)
    mid = 0.5 * (t.max() + t.min())
    out = {}
    for ph, cols in (("L", ok & (t > mid)), ("V", ok & (t < mid))):
        c = p[:, cols].mean(axis=1) if cols.any() else None
        out[ph] = None if c is None else (c.sum(), c / c.sum())
    return out


def test_fp32_sweep_instances_bulk_phases_at_equilibrium():
    """FP32 storage against FP64 at equilibrium on the benchmark sweep's own
    instances (C1/C3/nC10 flat slabs on their square grids; one instance of
    each size 64^2 ... 176^2, both precisions batched as timed), 2e6 steps:
    the residual over the last 1e5 steps at or below 1e-9, and every phase
    that has bulk sites in both runs (max_i |grad rt_i| / rt_i < 1e-4) within
    1e-4 relative density and 1e-3 absolute mole fraction.  The bulk is
    found by that criterion, not by fixed windows: a slab may settle one
    lattice site away from the other precision's (an equivalent
    equilibrium), and fixed windows then read interface tails."""
    capi = _capi()
    from paper_2306_10652_amd import batch
    from oracle.lbm import oracle_mixture
    specs = batch.ternary_specs(W.states()["ternary_sweep"])
    sizes = [sp["shape"][0] for sp in specs]
    pick = [sizes.index(n) for n in sorted(set(sizes))[:8]]
    sel = [specs[k] for k in pick]
    import torch
    a = batch.Sweep(sel, capi.FP32_STORAGE, stream=torch.cuda.Stream())
    b = batch.Sweep(sel, capi.FP64, stream=torch.cuda.Stream())
    # the two precisions side by side, one stream each
    W.run_side_by_side([a.step, b.step], 1900000)
    for sw in (a, b):
        for s in sw.sims:
            s.diagnostics()
    W.run_side_by_side([a.step, b.step], 100000)
    worst_rho, worst_x, compared, worst_res = 0.0, 0.0, 0, 0.0
    for sa, sb, sp in zip(a.sims, b.sims, sel):
        worst_res = max(worst_res, sa.diagnostics()["residual"], sb.diagnostics()["residual"])
        M = oracle_mixture(sp["comps"], sp["T"]).M
        pa, pb = _bulk_by_gradient(sa, M), _bulk_by_gradient(sb, M)
        for ph in ("L", "V"):
            if pa[ph] is None or pb[ph] is None:
                continue
            compared += 1
            worst_rho = max(worst_rho, abs(pa[ph][0] / pb[ph][0] - 1))
            worst_x = max(worst_x, float(np.max(np.abs(pa[ph][1] - pb[ph][1]))))
    report("fp32_vs_fp64_sweep_instances", instances=pick, phases=compared, rho_rel=worst_rho,
           x_abs=worst_x, residual=worst_res)
    a.close()
    b.close()
    assert worst_res <= 1e-9
    assert compared >= 12
    assert worst_rho <= 1e-4 and worst_x <= 1e-3


def test_full_size_sweep_sampled_parity():
    """The benchmark's batched sweep at full size (256 C1/C3/nC10 instances,
    64^2 ... 256^2, FP32 storage, one launch per step as timed): after 20
    batched steps, sampled instances (the first, a middle one, the largest
    and the last) against the oracle run alone, every density within the
    FP32-storage bar of 1e-4 relative."""
    capi = _capi()
    from paper_2306_10652_amd import batch
    from oracle.lbm import OracleLBM, oracle_mixture
    S = W.states()["ternary_sweep"]
    specs = batch.ternary_specs(S)
    sw = batch.Sweep(specs, capi.FP32_STORAGE)
    sw.step(20)
    big = int(np.argmax([np.prod(sp["shape"]) for sp in specs]))
    worst = 0.0
    for k in sorted({0, len(specs) // 2, big, len(specs) - 1}):
        sp = specs[k]
        o = OracleLBM(oracle_mixture(sp["comps"], sp["T"]), 0, sp["shape"], sp["rho"])
        o.run(20)
        g = sw.sims[k].read_moments(velocity=False)["rho"]
        e = float(np.max(np.abs(g - o.rho()) / np.abs(o.rho())))
        report("sweep_full_parity", instance=k, shape=sp["shape"], rho_rel=e)
        worst = max(worst, e)
    sw.close()
    assert worst <= 1e-4


def serving_requests(count=5, tol=1e-6, max_steps=4000):
    from paper_2306_10652_amd import serve
    reqs = serve.pool_requests(W.states()["serving_pool"], count, rate_hz=200.0, tol=tol,
                               max_steps=max_steps, max_n2d=96, max_n3d=20)
    return reqs


def test_server_results_match_oracle():
    """Requests served in the mix (D2Q9 and a D3Q19 one, FP32 storage,
    batched with each other) against the oracle run alone for the same
    number of steps: every density within 1e-4 relative."""
    capi = _capi()
    from paper_2306_10652_amd import serve
    from oracle.lbm import OracleLBM, oracle_mixture
    reqs = serve.pool_requests(W.states()["serving_pool"], 8, rate_hz=200.0, tol=1e-12,
                               max_steps=200, max_n2d=64, max_n3d=16)
    assert any(r.lattice == capi.D3Q19 for r in reqs)
    srv = serve.Server(8 << 30, chunk=100, keep_fields=True)
    done = srv.run(reqs)
    worst = 0.0
    for r in done:
        assert r.status == 0 and r.steps == 200
        o = OracleLBM(oracle_mixture(r.comps, r.T), r.lattice, r.shape, r.rho)
        o.run(r.steps)
        rho_o = o.rho()
        e = float(np.max(np.abs(r.result["rho"] - rho_o) / np.abs(rho_o)))
        report("serve_oracle", rid=r.rid, lattice=r.lattice, shape=r.shape, N=r.N, rho_rel=e)
        worst = max(worst, e)
    assert worst <= 1e-4


def test_server_alone_equals_mix_and_budget():
    capi = _capi()
    from paper_2306_10652_amd import serve
    alone = {}
    for r in serving_requests():
        r.arrival = 0.0
        srv = serve.Server(8 << 30, chunk=200, keep_fields=True)
        srv.run([r])
        alone[r.rid] = r
    mix = serving_requests()
    one = mix[0]
    budget = one.nbytes() + max(r.nbytes() for r in mix[1:]) + 1   # at most ~2 resident
    srv = serve.Server(budget, chunk=200, keep_fields=True)
    peak = [0]
    admit = srv._admit

    def watch(req, now):
        s = admit(req, now)
        peak[0] = max(peak[0], srv.used)
        return s
    srv._admit = watch
    done = srv.run(mix)
    assert peak[0] <= budget
    assert len(done) == len(mix)
    for r in done:
        a = alone[r.rid]
        report("serve_mix", rid=r.rid, steps=r.steps, alone_steps=a.steps,
               converged=r.converged, latency=r.finish_t - r.arrival)
        assert r.status == 0 and r.steps == a.steps
        assert np.array_equal(r.result["populations"], a.result["populations"])
    st = serve.latency_stats(done)
    nconv = sum(r.converged for r in done)
    assert st["requests"] == len(mix) and st["converged"] == nconv
    assert st["capped"] == len(mix) - nconv and st["failed"] == 0
    if nconv:
        assert st["p99_s"] >= st["p50_s"] > 0


def test_server_isolates_a_failing_request():
    """A request whose state turns non-finite (a NaN written into one
    population after admission) fails alone with ENONFINITE; the requests
    sharing the batched launches with it finish exactly as they do alone."""
    capi = _capi()
    from paper_2306_10652_amd import serve
    alone = {}
    for r in serving_requests(count=3):
        r.arrival = 0.0
        srv = serve.Server(8 << 30, chunk=200, keep_fields=True)
        srv.run([r])
        alone[r.rid] = r
    reqs = serving_requests(count=3)
    bad = serving_requests(count=1)[0]
    bad.rid = 99
    srv = serve.Server(8 << 30, chunk=200, keep_fields=True)
    admit = srv._admit

    def poison(req, now):
        slot = admit(req, now)
        if req.rid == 99:
            slot["sim"].poke(0, 0, 5, float("nan"))
        return slot
    srv._admit = poison
    done = srv.run(reqs + [bad])
    by = {r.rid: r for r in done}
    report("serve_isolation", bad_status=by[99].status, others=[by[r.rid].steps for r in reqs])
    assert by[99].status == 5
    for r in reqs:
        got = by[r.rid]
        assert got.status == 0 and got.steps == alone[r.rid].steps
        assert np.array_equal(got.result["populations"], alone[r.rid].result["populations"])
