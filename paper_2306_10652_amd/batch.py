"""Batched sweeps: many independent D2Q9 simulations (uneven grids, each its
own T, p and z) advanced with ONE fused launch per step through
``fuglbm_step_many``; runs of steps are replayed from a captured hipGraph
inside the library.

Also the read-out used to compare a sweep with a reference run: bulk
vapour / liquid windows of a flat slab (paper Section III.B: vapour at the
box edges, liquid in the middle).
"""
import numpy as np

from . import capi


def slab_windows(nx):
    """Vapour columns at the box edges and liquid columns at the centre of a
    slab with the liquid in the middle half (x in [nx/4, 3nx/4))."""
    q = max(1, nx // 16)
    vap = np.r_[0:q, nx - q:nx]
    liq = np.r_[nx // 2 - q:nx // 2 + q]
    return vap, liq


def bulk_phases(rho, M):
    """Bulk molar densities and mole fractions of both phases of a slab.
    rho: [N][nz][ny][nx] mass densities; M: lattice molar masses."""
    rt = rho / np.asarray(M)[:, None, None, None]
    nx = rho.shape[-1]
    vap, liq = slab_windows(nx)
    rv = rt[..., vap].mean(axis=(1, 2, 3))
    rl = rt[..., liq].mean(axis=(1, 2, 3))
    return dict(rho_V=rv.sum(), rho_L=rl.sum(), y=rv / rv.sum(), x=rl / rl.sum())


class Sweep:
    """A set of simulations stepped together.

    ``specs``: list of dicts with keys comps (component records with Tc, pc,
    omega, M), T, kij (or None), shape, rho (initial mass densities).
    """

    def __init__(self, specs, precision=capi.FP32_STORAGE, kappa_ref=0.02, tau=1.0,
                 stream=None):
        self.stream = stream
        self.mixtures, self.sims = [], []
        for sp in specs:
            mix = capi.Mixture.from_components(sp["comps"], sp["T"], sp.get("kij"),
                                               kappa_ref=kappa_ref, tau=tau)
            sim = capi.Simulation(mix, capi.D2Q9, precision, sp["shape"], sp["rho"],
                                  stream=stream)
            self.mixtures.append(mix)
            self.sims.append(sim)

    @property
    def sites(self):
        return sum(s.sites for s in self.sims)

    @property
    def csu_per_step(self):
        return sum(s.sites * s.N for s in self.sims)

    def step(self, nsteps):
        capi.step_many(self.sims, nsteps, self.stream)

    def step_sequential(self, nsteps):
        """The same work one simulation at a time (comparison baseline)."""
        for s in self.sims:
            s.step_n(nsteps, self.stream)

    def phases(self):
        out = []
        for s, m in zip(self.sims, self.mixtures):
            rho = s.read_moments(velocity=False)["rho"]
            out.append(bulk_phases(rho, m.molar_masses_lu()))
        return out

    def close(self):
        for s in self.sims:
            s.close()
        for m in self.mixtures:
            m.close()
        self.sims, self.mixtures = [], []


def ternary_specs(states, count=None):
    """Sweep specs from the stored ternary phase states (flat slabs)."""
    from inputs import fields as Fi
    comps = [_Comp(**c) for c in states["components"]]
    specs = []
    for inst in states["instances"][:count]:
        n = inst["n"]
        rho = Fi.slab(n, n, inst["rho_V"], inst["rho_L"], inst["S_V"])
        specs.append(dict(comps=comps, T=inst["T"], kij=None, shape=(n, n), rho=rho))
    return specs


class _Comp:
    def __init__(self, name, Tc, pc, omega, M):
        self.name, self.Tc, self.pc, self.omega, self.M = name, Tc, pc, omega, M
