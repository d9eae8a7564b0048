"""Pins of the oracle's diagnostics (no GPU): per-component mass, the
populations' momentum, the force-corrected momentum sum_r rho u, the
equilibrium residual and the status bits of a state.

Each expected value comes from something other than the oracle's own code:
* mass: the closed form sum_r rho_i of the field the state was made from,
  and its conservation by Eq. (1a)-(1c) (sum_a F_a = 0, sum_a (geq - g) = 0);
* momentum of hand-built populations: sum_a e_a g written out per direction;
* the force correction: on a periodic lattice the antisymmetric gradient
  stencil sums by parts, sum_r rt_i grad(psi_i) = -sum_r psi_i grad(rt_i),
  so sum_r (rho u - j) = (1/2) sum_i sum_r psi_i grad(rt_i), evaluated here
  with the test's own numpy stencil on the other factor;
* the residual of two hand-built states differing at one site;
* status bits of states outside the EOS domain.
"""
import numpy as np
import pytest

from tests import workloads as W
from oracle import lbm


def _direction_index(lattice):
    E, w = lbm.velocity_set(lattice)
    return E, w


def _fill(o, pops):
    """Set the oracle's populations from an array [N][Q][sites] in the
    oracle's own direction order."""
    N, Q, ns = pops.shape
    o.g[:] = pops.transpose(2, 0, 1).ravel()


@pytest.mark.parametrize("lattice,shape", [(0, (23, 17)), (1, (9, 8, 7))])
def test_mass_closed_form_and_conserved(lattice, shape, oracle_lib):
    wl = W.random_droplet(3, shape, seed=11, lattice=lattice)
    o = wl.oracle()
    d = o.diagnostics()
    want = np.array([np.sum(np.sort(r.ravel())) for r in np.asarray(wl.rho)])
    np.testing.assert_allclose(d["mass"], want, rtol=1e-14)
    o.run(40)
    d2 = o.diagnostics()
    np.testing.assert_allclose(d2["mass"], want, rtol=1e-13)
    assert d2["status"] == 0


@pytest.mark.parametrize("lattice,shape", [(0, (12, 10)), (1, (6, 5, 4))])
def test_population_momentum_of_hand_built_state(lattice, shape, oracle_lib):
    """Every direction gets its own random population: sum_r sum_i sum_a e_a g
    written out direction by direction.  On a uniform density field every
    gradient vanishes exactly, so the force-corrected momentum equals it."""
    wl = W.random_droplet(2, shape, seed=3, lattice=lattice)
    o = wl.oracle()
    E, w = _direction_index(lattice)
    Q = len(w)
    ns = int(np.prod(shape))
    rng = np.random.default_rng(7)
    pops = rng.uniform(0.0, 0.05, (2, Q, ns))
    # uniform total per component: rest population tops every site up to rho_i
    rho_i = np.array([0.9, 0.3])
    pops[:, 0, :] = rho_i[:, None] - (pops.sum(axis=1) - pops[:, 0, :])
    _fill(o, pops)
    d = o.diagnostics()
    want = np.zeros(3)
    for a in range(Q):
        for k in range(3):
            want[k] += E[a, k] * pops[:, a, :].sum()
    np.testing.assert_allclose(d["momentum_pop"], want, atol=1e-14 * pops.sum())
    np.testing.assert_allclose(d["momentum"], want, atol=1e-14 * pops.sum())
    np.testing.assert_allclose(d["mass"], rho_i * ns, rtol=1e-14)


def _grad_np(phi, lattice):
    """The isotropic gradient 3 sum_a w_a e_a phi(r + e_a) (the pairwise
    form summed over both members of a pair), periodic, on [z][y][x]."""
    E, w = lbm.velocity_set(lattice)
    out = np.zeros((3,) + phi.shape)
    for a in range(len(w)):
        sh = phi
        for k, ax in ((0, 2), (1, 1), (2, 0)):
            if E[a, k]:
                sh = np.roll(sh, -int(E[a, k]), axis=ax)
        for k in range(3):
            out[k] += 3.0 * w[a] * E[a, k] * sh
    return out


@pytest.mark.parametrize("lattice,shape", [(0, (23, 17)), (1, (9, 8, 7))])
def test_force_corrected_momentum_by_parts(lattice, shape, oracle_lib):
    """sum_r rho u - sum_r j = (1/2) sum_i sum_r F_i = (1/2) sum_i sum_r
    psi_i grad(rt_i): the gradient moved onto the molar density (summation
    by parts of the antisymmetric stencil on a periodic lattice)."""
    wl = W.random_droplet(3, shape, seed=21, lattice=lattice, noise=5e-2)
    o = wl.oracle()
    o.run(3)
    d = o.diagnostics()
    f = o.fields()
    M = o.mix.M
    rt = f["rho"] / M[:, None, None, None]
    corr = np.zeros(3)
    scale = 0.0
    for i in range(o.mix.N):
        gr = _grad_np(rt[i], lattice)
        for k in range(3):
            corr[k] += 0.5 * np.sum(f["psi"][i] * gr[k])
        scale += np.sum(np.abs(f["psi"][i] * gr))
    got = d["momentum"] - d["momentum_pop"]
    assert np.max(np.abs(corr)) > 1e-6 * scale       # the correction is not trivially zero
    np.testing.assert_allclose(got, corr, atol=1e-12 * scale)
    if lattice == 0:
        assert d["momentum"][2] == 0.0 and d["momentum_pop"][2] == 0.0


def test_residual_of_hand_built_pair(oracle_lib):
    """Two states made from fields that differ at one site of component 1 by
    delta: R = |delta| / (K sum_r rho_1(t)) (the later state's mass), the
    other components contribute 0; identical states give 0."""
    wl = W.random_droplet(3, (16, 12), seed=5)
    o = wl.oracle()
    g_prev = o.g.copy()
    rho = np.array(wl.rho, dtype=np.float64).copy()
    delta = 0.25 * rho[1, 0, 5, 7]
    rho[1, 0, 5, 7] += delta
    from oracle.lbm import OracleLBM
    o2 = OracleLBM(o.mix, 0, (16, 12), rho)
    K = 7
    d = o2.diagnostics(g_prev, K)
    want = abs(delta) / (K * rho[1].sum())
    assert abs(d["residual"] - want) <= 1e-13 * want
    d0 = o.diagnostics(g_prev, K)
    assert d0["residual"] == 0.0
    assert o.diagnostics(g_prev, 0)["residual"] == 0.0


def test_status_bits(oracle_lib):
    """A negative molar density sets bit 4; a site past the co-volume
    (b_m rt >= 1) sets bit 2; a finite in-domain state sets none."""
    wl = W.random_droplet(2, (8, 8), seed=2)
    o = wl.oracle()
    assert o.diagnostics()["status"] == 0
    rho = np.array(wl.rho, dtype=np.float64).copy()
    rho[0, 0, 3, 3] = -rho[0, 0, 3, 3]
    from oracle.lbm import OracleLBM
    assert OracleLBM(o.mix, 0, (8, 8), rho).diagnostics()["status"] & 4
    rho = np.array(wl.rho, dtype=np.float64).copy()
    b = o.mix.pr.b
    rho[:, 0, 2, 2] = 2.0 * o.mix.M / (b.sum())       # b_m rt = 2 at one site
    assert OracleLBM(o.mix, 0, (8, 8), rho).diagnostics()["status"] & 2
