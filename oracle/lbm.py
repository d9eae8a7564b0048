"""Python front of the CPU oracle LBM (``lbm_oracle.c``) plus the oracle's own
lattice-unit set-up of a mixture.

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.

``oracle_mixture`` follows the paper's unit anchoring (Section III.A: R, a, b
and M of the reference component fixed in lattice units) and the kappa
approximation of Eq. (6) (kappa_i = kappa_ref a_i / a_ref, with a_i the
attraction parameter without alpha, Eq. (7)).
"""
import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from . import thermo

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")
MAXC = 16

GCC_CMD = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
           "-std=c99", SRC, "-o", LIB, "-lm"]


def build_oracle(force=False):
    """Compile the oracle library (plain gcc, no GPU code)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        subprocess.check_call(GCC_CMD)
    return LIB


class OracleParams(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("N", ctypes.c_int),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("tau", ctypes.c_double), ("RT", ctypes.c_double),
                ("rho_c", ctypes.c_double),
                ("b", ctypes.c_double * MAXC), ("M", ctypes.c_double * MAXC),
                ("sqk", ctypes.c_double * MAXC),
                ("aij", ctypes.c_double * (MAXC * MAXC)),
                ("eos", ctypes.c_int), ("d1", ctypes.c_double), ("d2", ctypes.c_double)]

EOS_CODE = {"PR": 0, "SRK": 1, "vdW": 2}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(OracleParams)
        L.oracle_velocity_set.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
        L.oracle_equilibrium.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        L.oracle_forcing.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        L.oracle_ln_fugacity.argtypes = [pp, dp, dp, dp]
        L.oracle_ln_fugacity.restype = ctypes.c_int
        L.oracle_gradient.argtypes = [pp, dp, dp]
        L.oracle_laplacian.argtypes = [pp, dp, dp]
        L.oracle_init.argtypes = [pp, dp, dp]
        L.oracle_step.argtypes = [pp, dp, dp]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_run.argtypes = [pp, dp, ctypes.c_long]
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads.restype = ctypes.c_int
        L.oracle_run.restype = ctypes.c_int
        L.oracle_fields.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        L.oracle_fields.restype = ctypes.c_int
        L.oracle_diagnostics.argtypes = [pp, dp, dp, ctypes.c_long, dp, dp, dp, dp]
        L.oracle_diagnostics.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def velocity_set(lattice):
    e = (ctypes.c_int * 57)()
    w = (ctypes.c_double * 19)()
    Q = lib().oracle_velocity_set(lattice, e, w)
    E = np.array(e[:3 * Q], dtype=np.int64).reshape(Q, 3)
    return E, np.array(w[:Q])


@dataclass
class OracleMixture:
    """A mixture in lattice units, as the oracle sees it."""
    comps: list
    units: thermo.LatticeUnits
    pr: thermo.PRMixture        # lattice-unit cubic-EOS mixture (PR unless eos says otherwise)
    M: np.ndarray               # lattice molar masses
    sqk: np.ndarray             # sqrt(kappa_i)
    tau: float
    T_K: float

    @property
    def N(self):
        return len(self.comps)

    @property
    def RT(self):
        return self.pr.RT

    def lattice_constants(self):
        """[RT, then per component (b_i, (a alpha)_i, sqrt kappa_i, M_i), then
        the N x N matrix (a alpha)_ij], the layout the GPU library exports."""
        out = [self.RT]
        for i in range(self.N):
            out += [self.pr.b[i], self.pr.aalpha[i], self.sqk[i], self.M[i]]
        out += list(self.pr.aij.ravel())
        return np.array(out)


def oracle_mixture(comps, T_K, kij=None, ref=0, kappa_ref=0.02, a_lu=2.0 / 49.0,
                   b_lu=2.0 / 21.0, R_lu=1.0, tau=1.0, eos="PR"):
    """The paper's anchors (a_ref = 2/49, b_ref = 2/21, R = 1) by default,
    for every EOS."""
    units = thermo.LatticeUnits(comps[ref], a_lu, b_lu, R_lu, eos=eos)
    pr = units.mixture(comps, T_K, kij)
    M = units.molar_masses(comps)
    kappa = kappa_ref * pr.a / pr.a[ref]          # Eq. (6)-(8)
    return OracleMixture(list(comps), units, pr, M, np.sqrt(kappa), tau, T_K)


def make_params(mix, lattice, nx, ny, nz=1, rho_c=0.0):
    P = OracleParams()
    P.lattice = lattice
    P.N = mix.N
    P.nx, P.ny, P.nz = nx, ny, nz
    P.tau = mix.tau
    P.RT = mix.RT
    P.rho_c = rho_c
    P.eos = EOS_CODE[mix.pr.eos]
    P.d1, P.d2 = mix.pr.d1, mix.pr.d2
    for i in range(mix.N):
        P.b[i] = mix.pr.b[i]
        P.M[i] = mix.M[i]
        P.sqk[i] = mix.sqk[i]
        for j in range(mix.N):
            P.aij[i * MAXC + j] = mix.pr.aij[i, j]
    return P


class OracleLBM:
    """A simulation held by the oracle: populations g[site][i][alpha]."""

    def __init__(self, mix, lattice, shape, rho0, rho_c=0.0):
        nx, ny, nz = (tuple(shape) + (1, 1))[:3]
        self.mix = mix
        self.lattice = lattice
        self.nx, self.ny, self.nz = nx, ny, nz
        self.Q = 9 if lattice == 0 else 19
        self.P = make_params(mix, lattice, nx, ny, nz, rho_c)
        self.ns = nx * ny * nz
        rho0 = np.ascontiguousarray(np.asarray(rho0, dtype=np.float64).reshape(mix.N, self.ns))
        self.g = np.zeros(self.ns * mix.N * self.Q)
        lib().oracle_init(ctypes.byref(self.P), _dp(rho0), _dp(self.g))
        self.steps = 0
        self.status = 0

    def run(self, nsteps):
        self.status |= lib().oracle_run(ctypes.byref(self.P), _dp(self.g), int(nsteps))
        self.steps += int(nsteps)
        return self.status

    def fields(self):
        N, ns = self.mix.N, self.ns
        rho = np.zeros(N * ns)
        u = np.zeros(3 * ns)
        psi = np.zeros(N * ns)
        lnf = np.zeros(N * ns)
        F = np.zeros(N * 3 * ns)
        st = lib().oracle_fields(ctypes.byref(self.P), _dp(self.g), _dp(rho), _dp(u),
                                 _dp(psi), _dp(lnf), _dp(F))
        shp = (self.nz, self.ny, self.nx)
        return dict(rho=rho.reshape((N,) + shp), u=u.reshape((3,) + shp),
                    psi=psi.reshape((N,) + shp), lnf=lnf.reshape((N,) + shp),
                    F=F.reshape((N, 3) + shp), status=st)

    def rho(self):
        return self.fields()["rho"]

    def diagnostics(self, g_prev=None, K=0):
        """Mass per component, the populations' momentum, the force-corrected
        momentum sum_r rho u and the residual against g_prev (a copy of
        ``self.g`` taken K steps earlier), plus status bits."""
        N = self.mix.N
        mass = np.zeros(N)
        mp = np.zeros(3)
        mu = np.zeros(3)
        res = ctypes.c_double()
        gp = None if g_prev is None else np.ascontiguousarray(g_prev, dtype=np.float64)
        st = lib().oracle_diagnostics(ctypes.byref(self.P), _dp(self.g), _dp(gp), int(K),
                                      _dp(mass), _dp(mp), _dp(mu), ctypes.byref(res))
        return dict(mass=mass, momentum_pop=mp, momentum=mu, residual=res.value, status=st)

    def populations(self):
        """Populations as [N][Q][sites] (for comparisons only)."""
        return self.g.reshape(self.ns, self.mix.N, self.Q).transpose(1, 2, 0).copy()


def ln_fugacity_lu(mix, rt_vec):
    """ln f_i and p at one state, through the oracle C code (lattice units)."""
    P = make_params(mix, 0, 1, 1, 1)
    rt = np.ascontiguousarray(np.asarray(rt_vec, dtype=np.float64))
    lnf = np.zeros(mix.N)
    p = ctypes.c_double()
    st = lib().oracle_ln_fugacity(ctypes.byref(P), _dp(rt), _dp(lnf), ctypes.byref(p))
    return lnf, p.value, st


def equilibrium(lattice, rho, u, rho_c=0.0):
    E, w = velocity_set(lattice)
    out = np.zeros(len(w))
    uu = np.ascontiguousarray(np.resize(np.asarray(u, dtype=np.float64), 3))
    lib().oracle_equilibrium(lattice, float(rho), float(rho_c), _dp(uu), _dp(out))
    return out


def forcing(lattice, F, G, u):
    E, w = velocity_set(lattice)
    out = np.zeros(len(w))
    f3 = lambda v: np.ascontiguousarray(np.resize(np.asarray(v, dtype=np.float64), 3))
    Fv, Gv, uv = f3(F), f3(G), f3(u)
    lib().oracle_forcing(lattice, _dp(Fv), _dp(Gv), _dp(uv), _dp(out))
    return out


def gradient(lattice, phi):
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float64))
    shp = phi.shape[::-1] + (1,) * (3 - phi.ndim)
    P = OracleParams()
    P.lattice, P.N = lattice, 1
    P.nx, P.ny, P.nz = shp[0], shp[1], shp[2]
    out = np.zeros((3,) + phi.shape)
    lib().oracle_gradient(ctypes.byref(P), _dp(phi), _dp(out))
    return out


def laplacian(lattice, phi):
    phi = np.ascontiguousarray(np.asarray(phi, dtype=np.float64))
    shp = phi.shape[::-1] + (1,) * (3 - phi.ndim)
    P = OracleParams()
    P.lattice, P.N = lattice, 1
    P.nx, P.ny, P.nz = shp[0], shp[1], shp[2]
    out = np.zeros(phi.shape)
    lib().oracle_laplacian(ctypes.byref(P), _dp(phi), _dp(out))
    return out


def set_threads(n):
    """OpenMP threads of the oracle's loops (n <= 0: leave); returns the
    previous count."""
    return lib().oracle_set_threads(int(n))
