"""The allocation-free batched step (fuglbm_step_many_noalloc) against
fuglbm_step_many, through the C ABI: two calls in a row, the second on a
smaller batch (fewer, smaller simulations, so stale table entries of the
first call would show), both must leave every member bitwise where
fuglbm_step_many leaves it (the integer work tables and the per-site
arithmetic are the same, so the bar is bitwise)."""
import numpy as np
import pytest

from tests import workloads as W
from tests.test_gpu_parity import _capi, report

pytestmark = pytest.mark.gpu


def _make(capi, specs):
    out = []
    for N, shape, seed, prec, pre in specs:
        wl = W.random_droplet(N, shape, seed=seed)
        mix = wl.gpu_mixture()
        s = capi.Simulation(mix, 0, prec, shape, wl.rho)
        s._mix = mix
        if pre:
            s.step_n(pre)          # leaves the state in the other buffer
        out.append(s)
    return out


# (N, shape, seed, precision, steps taken alone before the batch); draws the
# oracle advances 45 steps without leaving the EOS domain
FIRST = [(3, (67, 45), 31, 0, 0), (3, (130, 19), 31, 0, 1), (3, (61, 23), 52, 1, 0),
         (5, (125, 17), 52, 0, 3), (2, (200, 9), 31, 1, 0), (10, (70, 21), 9, 0, 0)]
SECOND = [(3, (40, 21), 52, 0, 0), (2, (9, 5), 31, 1, 1)]


@pytest.mark.parametrize("order", ["first_then_second"])
def test_noalloc_matches_step_many(order):
    capi = _capi()
    for label, specs, steps in (("first", FIRST, 41), ("second", SECOND, 16)):
        ref = _make(capi, specs)
        got = _make(capi, specs)
        capi.step_many(ref, steps)
        capi.step_many_noalloc(got, steps)
        for k, (a, b) in enumerate(zip(ref, got)):
            ga, gb = a.read_populations(), b.read_populations()
            da, db = a.diagnostics(), b.diagnostics()
            report("noalloc", call=label, member=k, equal=bool(np.array_equal(ga, gb)),
                   step=db["step"])
            assert np.array_equal(ga, gb), (label, k)
            assert da["step"] == db["step"]
            assert db["status"] == 0
        for s in ref + got:
            s.close()


def test_noalloc_rejects_what_it_cannot_run():
    """A D3Q19 member, a repeated member and negative steps are EINVAL and
    launch nothing; an empty batch and zero steps change nothing."""
    capi = _capi()
    a = _make(capi, [(3, (40, 21), 52, 0, 0)])[0]
    wl3 = W.random_droplet(2, (9, 8, 7), seed=31, lattice=1)
    m3 = wl3.gpu_mixture()
    b = capi.Simulation(m3, 1, 0, wl3.shape, wl3.rho)
    g0 = a.read_populations()
    assert capi.fuglbm_step_many_noalloc([a, b], 3) == 1
    assert capi.fuglbm_step_many_noalloc([a, a], 3) == 1
    assert capi.fuglbm_step_many_noalloc([a], -1) == 1
    assert capi.fuglbm_step_many_noalloc([], 5) == 0
    assert capi.fuglbm_step_many_noalloc([a], 0) == 0
    assert np.array_equal(a.read_populations(), g0)
    assert a.diagnostics()["step"] == 0
