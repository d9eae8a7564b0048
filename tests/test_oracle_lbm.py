"""Pins of the oracle's lattice Boltzmann step (no GPU).

* Closed-form moments of the equilibrium Eq. (1b) (rho^c = 0) and of the
  forcing term Eq. (1c), from 4th-order lattice isotropy.
* Stencil symbols: grad of sin(k.r) and lap of cos(k.r) have closed forms.
* A uniform state at rest is a bitwise fixed point; per-component mass is
  conserved; a reflection- and transpose-symmetric droplet stays symmetric.
* Split invariance: one fluid written as two identical pseudo-components
  evolves exactly like the single-component run.
* A flat single-component interface relaxes to the Maxwell coexistence
  densities (paper Table IV case 1 reports the same agreement).
"""
import numpy as np
import pytest

from inputs import components as C
from inputs import fields as Fi
from oracle import thermo as th
from oracle import lbm

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("lattice", [0, 1])
def test_equilibrium_moments(lattice, oracle_lib):
    E, w = lbm.velocity_set(lattice)
    D = 2 if lattice == 0 else 3
    rng = np.random.default_rng(lattice)
    for _ in range(20):
        rho = rng.uniform(0.1, 5.0)
        u = np.zeros(3)
        u[:D] = rng.uniform(-0.1, 0.1, D)
        geq = lbm.equilibrium(lattice, rho, u)
        assert abs(geq.sum() - rho) < 1e-14 * rho
        np.testing.assert_allclose(E.T @ geq, rho * u, atol=1e-15)
        Pi = np.einsum("a,ab,ac->bc", geq, E, E)
        np.testing.assert_allclose(Pi, rho * np.outer(u, u), atol=1e-14)


@pytest.mark.parametrize("lattice", [0, 1])
def test_forcing_moments(lattice, oracle_lib):
    """sum F_a = 0, sum e F_a = F, sum e e F_a = uF + Fu + cs^2[(u.G) I + uG + Gu]."""
    E, w = lbm.velocity_set(lattice)
    D = 2 if lattice == 0 else 3
    rng = np.random.default_rng(10 + lattice)
    I = np.diag([1.0] * D + [0.0] * (3 - D))
    for _ in range(20):
        u, F, G = (np.zeros(3) for _ in range(3))
        u[:D] = rng.uniform(-0.1, 0.1, D)
        F[:D] = rng.uniform(-1, 1, D)
        G[:D] = rng.uniform(-1, 1, D)
        Fa = lbm.forcing(lattice, F, G, u)
        assert abs(Fa.sum()) < 1e-15
        np.testing.assert_allclose(E.T @ Fa, F, atol=1e-15)
        Pi = np.einsum("a,ab,ac->bc", Fa, E, E)
        want = (np.outer(u, F) + np.outer(F, u)
                + CS2 * ((u @ G) * I + np.outer(u, G) + np.outer(G, u)))
        np.testing.assert_allclose(Pi, want, atol=1e-14)


def test_velocity_sets(oracle_lib):
    for lattice, Q in ((0, 9), (1, 19)):
        E, w = lbm.velocity_set(lattice)
        assert E.shape == (Q, 3) and np.all(E[0] == 0)
        assert abs(w.sum() - 1) < 1e-15
        D = 2 if lattice == 0 else 3
        np.testing.assert_allclose(np.einsum("a,ab,ac->bc", w, E, E)[:D, :D],
                                   CS2 * np.eye(D), atol=1e-15)


@pytest.mark.parametrize("k", [1, 3, 7])
def test_stencil_symbols_d2q9(k, oracle_lib):
    """grad_d sin(kx x + ky y) and lap_d cos(.) against their lattice symbols:
    grad_d e^{ik.r} = i cs^-2 sum_a w_a e_a sin(k.e_a) e^{ik.r},
    lap_d  e^{ik.r} = 2 cs^-2 sum_a w_a (cos(k.e_a) - 1) e^{ik.r}."""
    n = 32
    kx, ky = 2 * np.pi * k / n, 2 * np.pi * (k + 1) / n
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ph = kx * x + ky * y
    # D2Q9 symbols written out (axis weight 1/9, diagonal 1/36)
    sx = 3 * (2 / 9 * np.sin(kx) + 1 / 18 * (np.sin(kx + ky) + np.sin(kx - ky)))
    sy = 3 * (2 / 9 * np.sin(ky) + 1 / 18 * (np.sin(kx + ky) - np.sin(kx - ky)))
    lap = 6 * (2 / 9 * (np.cos(kx) - 1 + np.cos(ky) - 1)
               + 1 / 18 * (np.cos(kx + ky) - 1 + np.cos(kx - ky) - 1))
    g = lbm.gradient(0, np.sin(ph))
    np.testing.assert_allclose(g[0], sx * np.cos(ph), atol=1e-13)
    np.testing.assert_allclose(g[1], sy * np.cos(ph), atol=1e-13)
    np.testing.assert_allclose(lbm.laplacian(0, np.cos(ph)), lap * np.cos(ph), atol=1e-13)


def test_stencils_exact_on_polynomials(oracle_lib):
    """Away from the periodic seam, grad_d is exact on linear fields and
    lap_d exact on quadratics (both lattices)."""
    for lattice, shape in ((0, (1, 24, 24)), (1, (12, 12, 12))):
        z, y, x = np.meshgrid(*[np.arange(s, dtype=float) for s in shape], indexing="ij")
        lin = 0.3 * x - 0.7 * y + (0.2 * z if lattice else 0)
        quad = 0.5 * x * x + 0.25 * y * y - 0.1 * x * y + (0.4 * z * z if lattice else 0)
        g = lbm.gradient(lattice, lin if lattice else lin[0])
        lp = lbm.laplacian(lattice, quad if lattice else quad[0])
        sl = (slice(1, -1),) * (3 if lattice else 2)
        np.testing.assert_allclose(g[0][sl], 0.3, atol=1e-12)
        np.testing.assert_allclose(g[1][sl], -0.7, atol=1e-12)
        want = 1.0 + 0.5 + (0.8 if lattice else 0)
        np.testing.assert_allclose(lp[sl], want, atol=1e-11)


def _droplet_setup(N=3, n=32, noise=True, lattice=0):
    comps = C.DROPLET_3[:N] if N <= 3 else C.N_ALKANES[:N]
    mix = lbm.oracle_mixture(comps, 250.0)
    rhoL = np.array([1.428, 3.167, 5.342])[:N]
    rhoV = np.array([0.837, 0.0943, 0.0141])[:N]
    f = Fi.droplet(n, n, rhoL, rhoV, n / 4.0)
    if noise:
        f = Fi.add_noise(f, 1e-3, 1)
    if lattice == 1:
        f = np.repeat(f, 8, axis=1)
    return mix, f


@pytest.mark.parametrize("lattice", [0, 1])
def test_uniform_state_is_bitwise_fixed_point(lattice, oracle_lib):
    mix, _ = _droplet_setup()
    shape = (12, 10, 6) if lattice else (16, 12)
    rho = Fi.uniform(shape[0], shape[1], [1.1, 0.4, 0.2], nz=shape[2] if lattice else 1)
    sim = lbm.OracleLBM(mix, lattice, shape, rho)
    g0 = sim.g.copy()
    sim.run(10)
    assert np.array_equal(sim.g, g0)


def test_mass_conservation_and_symmetry(oracle_lib):
    mix, f = _droplet_setup(noise=False)
    sim = lbm.OracleLBM(mix, 0, (32, 32), f)
    m0 = sim.rho().sum(axis=(1, 2, 3))
    sim.run(300)
    assert sim.status == 0
    r = sim.rho()[:, 0]
    np.testing.assert_allclose(r.sum(axis=(1, 2)), m0, rtol=1e-13)
    # droplet centred at (16, 16): symmetric under x -> 32 - x, y -> 32 - y, x <-> y
    flip = np.roll(r[:, :, ::-1], 1, axis=2)
    np.testing.assert_allclose(flip, r, rtol=1e-12)
    np.testing.assert_allclose(np.transpose(r, (0, 2, 1)), r, rtol=1e-12)


def test_mass_conservation_d3q19(oracle_lib):
    mix, f = _droplet_setup(N=2, n=12, lattice=1)
    sim = lbm.OracleLBM(mix, 1, (12, 12, 8), f)
    m0 = sim.rho().sum(axis=(1, 2, 3))
    sim.run(50)
    np.testing.assert_allclose(sim.rho().sum(axis=(1, 2, 3)), m0, rtol=1e-13)


def test_split_invariance(oracle_lib):
    """One PR fluid as two identical pseudo-components at a fixed fraction r
    per site evolves as r and (1 - r) times the single-component run: ln f_A
    differs from the pure value by ln r only, so every force scales by r."""
    c1 = C.TABLE_I["C1"]
    pure = lbm.oracle_mixture([c1], 170.0)
    pair = lbm.oracle_mixture([c1, c1], 170.0)
    n = 24
    rho = Fi.add_noise(Fi.droplet(n, n, [8.0], [0.7], 6.0), 1e-2, 3)
    r = 0.3
    s1 = lbm.OracleLBM(pure, 0, (n, n), rho)
    s2 = lbm.OracleLBM(pair, 0, (n, n), np.concatenate([r * rho, (1 - r) * rho]))
    s1.run(200)
    s2.run(200)
    a, b = s1.rho(), s2.rho()
    np.testing.assert_allclose(b[0], r * a[0], rtol=1e-11)
    np.testing.assert_allclose(b[1], (1 - r) * a[0], rtol=1e-11)


def test_flat_interface_relaxes_to_maxwell(oracle_lib):
    """Table II case 1 (pure C1, 177.24 K) on a 128 x 1 slab: bulk densities
    reach the Maxwell coexistence densities and the velocity decays to
    round-off (well-balanced scheme).  20 000 steps; the paper's 10^6-step
    run agrees to 2e-8 (Table IV), ours to 2e-5 after 20 000."""
    c1 = C.TABLE_I["C1"]
    mix = lbm.oracle_mixture([c1], 177.24)
    ps, rV, rL = th.maxwell(mix.pr)
    f = Fi.slab(128, 1, [0.98 * rV], [1.02 * rL], 0.5)
    sim = lbm.OracleLBM(mix, 0, (128, 1), f)
    sim.run(20000)
    fl = sim.fields()
    rt = fl["rho"][0, 0, 0] / mix.M[0]
    assert abs(rt[0] / rV - 1) < 2e-5
    assert abs(rt[64] / rL - 1) < 2e-5
    assert np.abs(fl["u"]).max() < 1e-9


@pytest.mark.parametrize("eos", ["SRK", "vdW"])
def test_flat_interface_relaxes_to_maxwell_other_cubics(oracle_lib, eos):
    """The same C1 slab (177.24 K, the paper's anchors) with the SRK or vdW
    equation of state in place of PR: the bulk densities (even windows)
    reach that EOS's own Maxwell densities and u decays to round-off."""
    c1 = C.TABLE_I["C1"]
    mix = lbm.oracle_mixture([c1], 177.24, eos=eos)
    ps, rV, rL = th.maxwell(mix.pr)
    f = Fi.slab(128, 1, [0.98 * rV], [1.02 * rL], 0.5)
    sim = lbm.OracleLBM(mix, 0, (128, 1), f)
    sim.run(20000)
    fl = sim.fields()
    rt = fl["rho"][0, 0, 0] / mix.M[0]
    assert abs(rt[0:4].mean() / rV - 1) < 2e-5
    assert abs(rt[62:66].mean() / rL - 1) < 2e-5
    assert np.abs(fl["u"]).max() < 1e-9


@pytest.mark.parametrize("eta", [0.1, 0.3])
def test_linear_acoustics_frequency(oracle_lib, eta):
    """A small density wave (amplitude 1e-6, wavelength 64) on a uniform
    supercritical C1 state (250 K, b rt0 = eta): linearising Eq. (1)-(5)
    about it gives an oscillator of frequency
        w0^2 = (1/M) [ (dp/drt)_T k^2 + kappa rt0 k^4 ],
    (continuity, momentum with the force -rt grad psi, and Gibbs-Duhem
    rt dmu = dp), with k^2 the lattice Laplacian's symbol 4 sin^2(pi/64).
    The wave's amplitude is fitted to A exp(-G t) cos(w t + phi) and
    w0^2 = w^2 + G^2 must match within 1e-3.  This pins the pressure the
    scheme carries: an equilibrium that kept c_s^2 rho, a wrong force sign
    or a dropped kappa term fails it."""
    from scipy.optimize import curve_fit
    c1 = C.TABLE_I["C1"]
    mix = lbm.oracle_mixture([c1], 250.0)
    rt0 = eta / mix.pr.b[0]
    M = mix.M[0]
    n = 64
    x = np.arange(n)
    f = (M * rt0 * (1 + 1e-6 * np.cos(2 * np.pi * x / n))).reshape(1, 1, 1, n)
    sim = lbm.OracleLBM(mix, 0, (n, 1), f)
    amp = []
    for _ in range(1500):
        r = sim.rho().reshape(-1)
        amp.append(np.sum((r - r.mean()) * np.cos(2 * np.pi * x / n)))
        sim.run(1)
    amp = np.array(amp) / amp[0]
    h = 1e-7 * rt0
    dpdr = (mix.pr.pressure_rho([rt0 + h]) - mix.pr.pressure_rho([rt0 - h])) / (2 * h)
    k2 = 4 * np.sin(np.pi / n) ** 2
    w_th = np.sqrt((dpdr * k2 + mix.sqk[0] ** 2 * rt0 * k2 ** 2) / M)
    model = lambda t, A, G, w, ph: A * np.exp(-G * t) * np.cos(w * t + ph)
    (A, G, w, ph), _ = curve_fit(model, np.arange(len(amp)), amp, p0=[1.0, 1e-3, w_th, 0.0])
    assert G > 0
    assert abs(np.sqrt(w * w + G * G) / w_th - 1) < 1e-3


def test_d3q19_reduces_to_d2q9_on_a_one_dimensional_field(oracle_lib):
    """A field that varies along x only: D2Q9 and D3Q19 both reduce to the
    same three-velocity lattice along x (weights 2/3, 1/6, 1/6; the same
    isotropic second-order forcing), so the two oracles give the same
    densities.  Pins the D3Q19 velocity set, weights and the D-dependent
    forcing term against the D2Q9 ones."""
    comps, T, _ = C.table_ii_components(3)
    mix = lbm.oracle_mixture(comps, T)
    st = Fi.load_phase_states()["vle3"]
    f2 = Fi.slab(64, 1, st["rho_V"], st["rho_L"], 0.5)
    a = lbm.OracleLBM(mix, 0, (64, 1), f2)
    b = lbm.OracleLBM(mix, 1, (64, 1, 1), f2)      # [N][nz=1][ny=1][nx]
    a.run(2000)
    b.run(2000)
    ra = a.rho().reshape(len(comps), -1)
    rb = b.rho().reshape(len(comps), -1)
    assert np.max(np.abs(ra - rb)) / np.max(np.abs(ra)) < 1e-12


def _drop3d(n=10, seed=7):
    """Two components, an off-centre spherical drop (no symmetry of the
    cube maps it to itself) with seeded noise, [N][nz][ny][nx]."""
    rhoL = np.array([1.428, 3.167])
    rhoV = np.array([0.837, 0.0943])
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = np.sqrt((x - 4.3) ** 2 + (y - 5.6) ** 2 + (z - 3.2) ** 2)
    prof = 0.5 * (1.0 - np.tanh((d - 3.0) / 2.0))
    f = rhoV[:, None, None, None] + (rhoL - rhoV)[:, None, None, None] * prof[None]
    return Fi.add_noise(f, 1e-3, seed)


def test_d3q19_commutes_with_the_cube_symmetries(oracle_lib):
    """D3Q19 (velocity set, weights, stencils, forcing) is invariant under
    the symmetries of the cube, so on a genuinely three-dimensional field
    with none of them, stepping a relabelled field equals relabelling the
    stepped one: a cyclic permutation of the axes and a reflection of each
    axis, after 30 steps.  One wrong lattice vector or weight among the 18
    moving directions breaks one of these."""
    mix, _ = _droplet_setup(N=2)
    f = _drop3d()
    n = f.shape[-1]

    def run(field):
        sim = lbm.OracleLBM(mix, 1, (n, n, n), np.ascontiguousarray(field))
        sim.run(30)
        assert sim.status == 0
        return sim.rho()

    base = run(f)
    assert np.max(np.abs(base - f)) > 1e-3                   # the field did evolve
    cyc = lambda a: np.transpose(a, (0, 2, 3, 1))          # relabel (z, y, x) -> (y, x, z)
    np.testing.assert_allclose(run(cyc(f)), cyc(base), rtol=1e-12, atol=0)
    for ax in (1, 2, 3):                                      # r -> -r along one axis
        refl = lambda a, ax=ax: np.roll(np.flip(a, axis=ax), 1, axis=ax)
        np.testing.assert_allclose(run(refl(f)), refl(base), rtol=1e-12, atol=0)


def test_d3q19_flat_interface_relaxes_to_maxwell(oracle_lib):
    """Table II case 1 on a 128 x 1 x 1 D3Q19 slab: the bulk densities reach
    the Maxwell coexistence densities (even windows) with u at round-off."""
    c1 = C.TABLE_I["C1"]
    mix = lbm.oracle_mixture([c1], 177.24)
    ps, rV, rL = th.maxwell(mix.pr)
    f = Fi.slab(128, 1, [0.98 * rV], [1.02 * rL], 0.5).reshape(1, 1, 1, 128)
    sim = lbm.OracleLBM(mix, 1, (128, 1, 1), f)
    sim.run(20000)
    fl = sim.fields()
    rt = fl["rho"].reshape(-1) / mix.M[0]
    assert abs(rt[0:4].mean() / rV - 1) < 2e-5
    assert abs(rt[62:66].mean() / rL - 1) < 2e-5
    assert np.abs(fl["u"]).max() < 1e-9
