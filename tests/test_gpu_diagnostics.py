"""Diagnostics of the GPU library (mass, force-corrected and population
momentum, residual, status) against the oracle's diagnostics of the same
state, through the C ABI, on both lattices and in both precisions.

Bars.  Mass: 1e-12 relative in both precisions (FP32 storage keeps every
component's mass to FP64 rounding, and both sides start from the same
field).  Momentum: the two sums differ by the populations' differences, so
the bar is absolute, relative to the total mass sum_r sum_i rho_i: 1e-12
in FP64, 1e-5 with FP32 storage (the stored moving populations carry
~6e-8 relative rounding each).  Residual: 1e-9 relative in FP64, 1e-4 with
FP32 storage (the FP32-storage density bar).
"""
import numpy as np
import pytest

from tests import workloads as W
from tests.test_gpu_parity import _capi, report

pytestmark = pytest.mark.gpu

# seeds: draws the oracle advances 33 steps without leaving the EOS domain
CASES = [(0, (67, 45), 3, 31), (0, (130, 19), 10, 9), (0, (9, 5), 1, 31),
         (1, (20, 18, 16), 3, 31), (1, (33, 9, 7), 5, 52)]


def _compare(dg, do, total_mass, precision, D, label):
    mtol = 1e-12
    ptol = (1e-12 if precision == 0 else 1e-5) * total_mass
    rtol = 1e-9 if precision == 0 else 1e-4
    em = float(np.max(np.abs(dg["mass"] - do["mass"]) / do["mass"]))
    ep = float(np.max(np.abs(dg["momentum"][:D] - do["momentum"][:D])))
    epp = float(np.max(np.abs(dg["momentum_pop"][:D] - do["momentum_pop"][:D])))
    er = abs(dg["residual"] - do["residual"]) / max(do["residual"], 1e-300)
    report(label, mass=em, mom=ep / total_mass, mom_pop=epp / total_mass, res=er,
           res_val=do["residual"])
    assert em <= mtol
    assert ep <= ptol and epp <= ptol
    if do["residual"] > 0:
        assert er <= rtol
    else:
        assert dg["residual"] == 0.0
    assert dg["status"] == do["status"] == 0
    assert np.all(dg["momentum"][D:] == 0.0)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("lattice,shape,N,seed", CASES)
def test_diagnostics_against_oracle(lattice, shape, N, seed, precision):
    """State after t0 steps (first call: residual 0), then after K more
    (residual over the K steps), GPU vs oracle."""
    capi = _capi()
    wl = W.random_droplet(N, shape, seed=seed, lattice=lattice)
    mix = wl.gpu_mixture()
    sim = capi.Simulation(mix, lattice, precision, wl.shape, wl.rho)
    o = wl.oracle()
    D = 2 if lattice == 0 else 3
    total = float(np.sum(wl.rho))
    t0, K = 20, 13
    sim.step_n(t0)
    assert o.run(t0) == 0
    g0 = o.g.copy()
    _compare(sim.diagnostics(), o.diagnostics(), total, precision, D,
             "diag_t0 lat=%d N=%d prec=%d" % (lattice, N, precision))
    sim.step_n(K)
    assert o.run(K) == 0
    _compare(sim.diagnostics(), o.diagnostics(g0, K), total, precision, D,
             "diag_tK lat=%d N=%d prec=%d" % (lattice, N, precision))
    sim.close()


def test_diagnostics_bitwise_reproducible():
    """The same state gives bitwise the same diagnostics however it was
    reached (batched or alone, either fused variant) and on a repeat."""
    capi = _capi()
    wls = [W.droplet64(seed=s) for s in (1, 2)]
    alone = []
    for wl in wls:
        mix = wl.gpu_mixture()
        s = capi.Simulation(mix, 0, 0, wl.shape, wl.rho)
        s.set_tuning(2, 4)
        s.diagnostics()
        s.step_n(50)
        alone.append(s.diagnostics())
        s._mix = mix
    mixes = [wl.gpu_mixture() for wl in wls]
    batch = [capi.Simulation(m, 0, 0, wl.shape, wl.rho) for m, wl in zip(mixes, wls)]
    for s in batch:
        s.diagnostics()
    capi.step_many(batch, 50)
    for s, ref in zip(batch, alone):
        d = s.diagnostics()
        for k in ("mass", "momentum", "momentum_pop"):
            assert np.array_equal(d[k], ref[k]), k
        assert d["residual"] == ref["residual"]


def test_diagnostics_headline_field_fp64():
    """The 1024 x 1024 ten-component field after 3 fused steps in its
    benchmark launch configuration: GPU diagnostics against the oracle's."""
    capi = _capi()
    wl = W.spinodal10()
    mix = wl.gpu_mixture()
    sim = capi.Simulation(mix, 0, 0, wl.shape, wl.rho)
    o = wl.oracle()
    sim.diagnostics()
    g0 = o.g.copy()
    sim.step_n(3)
    assert o.run(3) == 0
    _compare(sim.diagnostics(), o.diagnostics(g0, 3), float(np.sum(wl.rho)), 0, 2,
             "diag_spinodal10")
    sim.close()
