"""Peng-Robinson thermodynamics for the CPU oracle (FP64, plain NumPy).

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU-baseline
leg of the benchmark may import anything under ``oracle/``; the GPU library
never does, and this module shares no code with it.

Contents, each following the paper's Section II.C unless noted:

* ``alpha``                 -- the alpha(omega, T_r) correlation (two branches,
                               split at omega = 0.49); Soave's for SRK.
* ``PRMixture``             -- a_i, b_i, alpha_i, vdW mixing rules Eq. (10)-(11),
                               pressure Eq. (9), the cubic in Z obtained from
                               Eq. (9), ln phi_i exactly as printed in Eq. (12);
                               with ``eos="SRK"`` or ``"vdW"`` the same for those
                               cubics (table ``EOS``).
* ``LatticeUnits``          -- conversion to lattice units by fixing R, a, b and M
                               of a reference component (Section III.A).
* ``flash`` / ``maxwell``   -- textbook two-phase flash (Wilson start,
                               Rachford-Rice, successive substitution) and the
                               pure-component equal-area (equal-fugacity)
                               construction.  The paper uses a flash but does not
                               print its algorithm; these are written from the
                               thermodynamics, not from any listing.
* ``stability``             -- Michelsen's tangent-plane (TPD) stability test
                               of a feed at (T, p): stationary points of the
                               tangent-plane distance by successive substitution
                               from vapour- and liquid-like Wilson trials.
* ``flash3``                -- the three-phase flash of the three-phase case
                               (Section III.D): multiphase Rachford-Rice and
                               successive substitution, written from the same
                               thermodynamics (the paper used an external code).
"""
import math
from dataclasses import dataclass

import numpy as np

OMEGA_A = 0.457235529          # Section II.C, a_i prefactor
OMEGA_B = 0.077796074          # Section II.C, b_i prefactor
R_SI = 8.314462618             # J / (mol K)
BAR = 1.0e5                    # Pa
SQRT2 = math.sqrt(2.0)


# The cubic equations of state the oracle knows, written
#     p = RT / (v - b) - (a alpha) / ((v + d1 b)(v + d2 b)),
# with the prefactors of a = Omega_a R^2 Tc^2 / pc and b = Omega_b R Tc / pc
# that put the critical point at (Tc, pc).  PR is the paper's (Section II.C);
# Soave-Redlich-Kwong and van der Waals are the textbook alternatives the
# fugacity formulation admits unchanged (Section I: any multicomponent EOS).
_CBRT2 = 2.0 ** (1.0 / 3.0)
EOS = {
    "PR": dict(d1=1.0 + SQRT2, d2=1.0 - SQRT2, omega_a=OMEGA_A, omega_b=OMEGA_B),
    "SRK": dict(d1=1.0, d2=0.0, omega_a=1.0 / (9.0 * (_CBRT2 - 1.0)),
                omega_b=(_CBRT2 - 1.0) / 3.0),
    "vdW": dict(d1=0.0, d2=0.0, omega_a=27.0 / 64.0, omega_b=1.0 / 8.0),
}


def alpha(omega, Tr, eos="PR"):
    """alpha_i(T).  PR: the correlation of Section II.C, first branch for
    omega <= 0.49.  SRK: Soave's m = 0.480 + 1.574 w - 0.176 w^2.  vdW: 1."""
    omega = np.asarray(omega, dtype=np.float64)
    Tr = np.asarray(Tr, dtype=np.float64)
    if eos == "vdW":
        return np.ones(np.broadcast(omega, Tr).shape)
    if eos == "SRK":
        m = 0.480 + 1.574 * omega - 0.176 * omega ** 2
    else:
        m_low = 0.374640 + 1.54226 * omega - 0.26992 * omega ** 2
        m_high = (0.379642 + 1.48503 * omega - 0.164423 * omega ** 2
                  + 0.016666 * omega ** 3)
        m = np.where(omega <= 0.49, m_low, m_high)
    return (1.0 + m * (1.0 - np.sqrt(Tr))) ** 2


class PRMixture:
    """Cubic-EOS mixture at a fixed temperature, in any consistent units;
    Peng-Robinson (the paper's) unless ``eos`` names SRK or vdW.

    Parameters are per-component critical constants expressed in the same
    unit system as ``R`` and ``T`` (SI by default).  ``kij`` is the binary
    interaction matrix (the paper writes it delta_ij, Eq. (10)).
    """

    def __init__(self, Tc, pc, omega, T, kij=None, R=R_SI, eos="PR"):
        self.Tc = np.asarray(Tc, dtype=np.float64)
        self.pc = np.asarray(pc, dtype=np.float64)
        self.omega = np.asarray(omega, dtype=np.float64)
        self.N = self.Tc.size
        self.T = float(T)
        self.R = float(R)
        self.RT = self.R * self.T
        self.eos = eos
        e = EOS[eos]
        self.d1, self.d2 = e["d1"], e["d2"]
        self.a = e["omega_a"] * self.R ** 2 * self.Tc ** 2 / self.pc
        self.b = e["omega_b"] * self.R * self.Tc / self.pc
        self.alpha = alpha(self.omega, self.T / self.Tc, eos)
        self.aalpha = self.a * self.alpha
        k = np.zeros((self.N, self.N)) if kij is None else np.asarray(kij, dtype=np.float64)
        self.kij = k
        # (a alpha)_ij = sqrt((a alpha)_i (a alpha)_j) (1 - delta_ij), Eq. (10)
        self.aij = np.sqrt(np.outer(self.aalpha, self.aalpha)) * (1.0 - k)

    # -- mixing rules -----------------------------------------------------
    def mix(self, x):
        """b_m (Eq. 11), S_i = sum_j x_j (a alpha)_ij and (a alpha)_m (Eq. 10)."""
        x = np.asarray(x, dtype=np.float64)
        bm = float(x @ self.b)
        S = self.aij @ x
        am = float(x @ S)
        return bm, am, S

    # -- Eq. (9) ----------------------------------------------------------
    def pressure(self, x, v):
        """p = RT/(v - b_m) - (a alpha)_m / ((v + d1 b_m)(v + d2 b_m));
        for PR the denominator is v^2 + 2 b_m v - b_m^2 (Eq. (9))."""
        bm, am, _ = self.mix(x)
        return self.RT / (v - bm) - am / ((v + self.d1 * bm) * (v + self.d2 * bm))

    def pressure_rho(self, rho_molar):
        """Pressure from a vector of component molar densities."""
        rho_molar = np.asarray(rho_molar, dtype=np.float64)
        rt = rho_molar.sum()
        return self.pressure(rho_molar / rt, 1.0 / rt)

    # -- cubic in Z ---------------------------------------------------------
    def AB(self, x, p):
        bm, am, _ = self.mix(x)
        return am * p / self.RT ** 2, bm * p / self.RT

    def z_roots(self, x, p):
        """Real roots Z > B of the EOS rewritten with v = Z RT / p, ascending:
        with u = d1 + d2, w = d1 d2,

        Z^3 - (1 + B - uB) Z^2 + (A + wB^2 - uB - uB^2) Z - (AB + wB^2 + wB^3) = 0,

        for PR (u = 2, w = -1) Z^3 - (1 - B) Z^2 + (A - 3B^2 - 2B) Z -
        (AB - B^2 - B^3) = 0.  Each root is polished by Newton steps on the
        same polynomial.
        """
        A, B = self.AB(x, p)
        u, w = self.d1 + self.d2, self.d1 * self.d2
        c = [1.0, -(1.0 + B - u * B), A + w * B * B - u * B - u * B * B,
             -(A * B + w * B * B + w * B ** 3)]
        r = np.roots(c)
        out = []
        for z in r:
            if abs(z.imag) > 1e-7 * max(1.0, abs(z.real)):
                continue
            z = z.real
            for _ in range(6):
                f = ((z + c[1]) * z + c[2]) * z + c[3]
                df = (3.0 * z + 2.0 * c[1]) * z + c[2]
                if df == 0.0:
                    break
                z -= f / df
            if z > B:
                out.append(z)
        return sorted(out), A, B

    # -- Eq. (12) -----------------------------------------------------------
    def ln_phi(self, x, Z, p):
        """ln(f_i / (x_i p)).  PR: exactly the printed form of Eq. (12).
        SRK: the same form with its own d1, d2,
            (b_i/b_m)(Z - 1) - ln(Z - B)
            - A / (B (d1 - d2)) (2 S_i / a_m - b_i / b_m) ln[(Z + d1 B)/(Z + d2 B)].
        vdW (d1 = d2 = 0), the textbook expression
            b_i / (v - b_m) - ln(Z - B) - 2 S_i / (RT v)."""
        x = np.asarray(x, dtype=np.float64)
        bm, am, S = self.mix(x)
        v = Z * self.RT / p
        term2 = -math.log((v - bm) * p / self.RT)
        if self.eos == "vdW":
            return self.b / (v - bm) + term2 - 2.0 * S / (self.RT * v)
        term1 = self.b / bm * (p * v / self.RT - 1.0)
        if self.eos == "PR":
            coef = am / (2.0 * SQRT2 * bm * self.RT)
            bracket = self.b / bm - 2.0 / am * S
            lnr = math.log((v + (1.0 + SQRT2) * bm) / (v + (1.0 - SQRT2) * bm))
            return term1 + term2 + coef * bracket * lnr
        coef = am / ((self.d1 - self.d2) * bm * self.RT)
        bracket = self.b / bm - 2.0 / am * S
        lnr = math.log((v + self.d1 * bm) / (v + self.d2 * bm))
        return term1 + term2 + coef * bracket * lnr

    def ln_fugacity(self, x, Z, p):
        """ln f_i = ln(x_i p) + ln phi_i."""
        return np.log(np.asarray(x) * p) + self.ln_phi(x, Z, p)

    def ln_fugacity_rho(self, rho_molar):
        """ln f_i at a state given by its molar densities (requires p > 0)."""
        rho_molar = np.asarray(rho_molar, dtype=np.float64)
        rt = rho_molar.sum()
        x = rho_molar / rt
        p = self.pressure(x, 1.0 / rt)
        Z = p / (rt * self.RT)
        return self.ln_fugacity(x, Z, p)

    def phase(self, x, p, which):
        roots, _, _ = self.z_roots(x, p)
        if not roots:
            raise ValueError("no admissible cubic root")
        Z = roots[0] if which == "L" else roots[-1]
        return Z, self.ln_phi(x, Z, p)


# ---------------------------------------------------------------------------
# Flash (textbook: Wilson, Rachford-Rice, successive substitution)
# ---------------------------------------------------------------------------

def wilson_K(mix, p):
    """Wilson correlation: K_i = (pc_i / p) exp[5.373 (1 + w_i)(1 - Tc_i / T)]."""
    return mix.pc / p * np.exp(5.373 * (1.0 + mix.omega) * (1.0 - mix.Tc / mix.T))


def rachford_rice(z, K, tol=1e-15, maxit=200):
    """Vapour fraction beta solving sum z_i (K_i - 1) / (1 + beta (K_i - 1)) = 0.

    Safeguarded Newton on the open bracket (1/(1-K_max), 1/(1-K_min)); the
    result may fall outside [0, 1] (negative flash).  Returns None when all
    K_i are on one side of 1 (no root).
    """
    z = np.asarray(z, dtype=np.float64)
    K = np.asarray(K, dtype=np.float64)
    if K.max() <= 1.0 or K.min() >= 1.0:
        return None
    lo = 1.0 / (1.0 - K.max())
    hi = 1.0 / (1.0 - K.min())
    km1 = K - 1.0

    def g(beta):
        d = 1.0 + beta * km1
        return float(np.sum(z * km1 / d)), float(-np.sum(z * km1 * km1 / (d * d)))

    beta = 0.5 * (lo + hi)
    if 0.0 < lo < 1.0 or 0.0 < hi < 1.0 or (lo < 0.5 < hi):
        beta = min(max(0.5, lo + 1e-12), hi - 1e-12)
    for _ in range(maxit):
        f, df = g(beta)
        if f > 0.0:
            lo = beta
        else:
            hi = beta
        step = -f / df if df != 0.0 else 0.0
        nb = beta + step
        if not (lo < nb < hi):
            nb = 0.5 * (lo + hi)
        if abs(nb - beta) <= tol * max(1.0, abs(nb)):
            beta = nb
            break
        beta = nb
    return beta


def min_gibbs_phase(mix, x, p):
    """The cubic root of a single phase of composition x at (T, p) with the
    lowest molar Gibbs energy, i.e. the smallest sum_i x_i ln phi_i (the
    stable root when the cubic has three): returns (Z, ln phi)."""
    roots, _, _ = mix.z_roots(x, p)
    if not roots:
        raise ValueError("no admissible cubic root")
    best = None
    for Z in (roots[0], roots[-1]):
        lp = mix.ln_phi(x, Z, p)
        g = float(np.asarray(x) @ lp)
        if best is None or g < best[0]:
            best = (g, Z, lp)
    return best[1], best[2]


@dataclass
class StabilityResult:
    stable: bool          # no trial phase lowers the Gibbs energy
    tm_min: float         # smallest tangent-plane distance at a non-trivial stationary point
    w: np.ndarray         # composition of that trial phase (z if only trivial ones)
    trials: list          # (tm, w, trivial) of the vapour- and liquid-like searches


def stability(mix, z, p, tol=1e-12, maxit=5000, tm_tol=1e-10):
    """Michelsen's tangent-plane stability test of a feed z at (T, p).

    With d_i = ln z_i + ln phi_i(z) (the feed's stable root), the modified
    tangent-plane distance of a trial phase of mole numbers W is
        tm(W) = 1 + sum_i W_i (ln W_i + ln phi_i(w) - d_i - 1),  w = W / sum W,
    whose stationary points satisfy ln W_i = d_i - ln phi_i(w); there
    tm = 1 - sum W.  Two searches by successive substitution on that
    condition start from the Wilson vapour-like (W = z K) and liquid-like
    (W = z / K) trials.  The feed is unstable (splits into two phases) when
    a search ends at a non-trivial stationary point (w != z) with tm < 0.
    """
    z = np.asarray(z, dtype=np.float64)
    z = z / z.sum()
    _, lpz = min_gibbs_phase(mix, z, p)
    d = np.log(z) + lpz
    K = wilson_K(mix, p)
    trials = []
    for W0 in (z * K, z / K):
        lnW = np.log(W0)
        trivial = False
        for _ in range(maxit):
            W = np.exp(lnW)
            w = W / W.sum()
            _, lpw = min_gibbs_phase(mix, w, p)
            new = d - lpw
            step = np.max(np.abs(new - lnW))
            lnW = new
            if np.max(np.abs(w - z)) < 1e-7:
                trivial = True
                break
            if step < tol:
                break
        W = np.exp(lnW)
        w = W / W.sum()
        trivial = trivial or np.max(np.abs(w - z)) < 1e-7
        trials.append((1.0 - float(W.sum()), w, trivial))
    nontriv = [t for t in trials if not t[2]]
    if nontriv:
        tm, w, _ = min(nontriv, key=lambda t: t[0])
    else:
        tm, w = 0.0, z
    return StabilityResult(bool(tm >= -tm_tol), float(tm), w, trials)


@dataclass
class FlashResult:
    beta: float           # vapour mole fraction
    x: np.ndarray         # liquid composition
    y: np.ndarray         # vapour composition
    ZL: float
    ZV: float
    rhoL: float           # liquid molar density (units of the mixture)
    rhoV: float           # vapour molar density
    iterations: int
    converged: bool
    two_phase: bool


def flash(mix, z, p, K0=None, tol=1e-13, maxit=20000):
    """Isothermal two-phase flash at (T, p, z) by successive substitution.

    Stops when max |delta ln K| < tol.  ``two_phase`` is False when the
    Rachford-Rice root is outside (0, 1) or K collapses to 1 (trivial
    solution).
    """
    z = np.asarray(z, dtype=np.float64)
    z = z / z.sum()
    K = wilson_K(mix, p) if K0 is None else np.asarray(K0, dtype=np.float64).copy()
    lnK = np.log(K)
    converged = False
    beta = None
    x = y = z
    ZL = ZV = float("nan")
    it = 0
    for it in range(1, maxit + 1):
        beta = rachford_rice(z, K)
        if beta is None:
            break
        x = z / (1.0 + beta * (K - 1.0))
        y = K * x
        x = x / x.sum()
        y = y / y.sum()
        ZL, lpl = mix.phase(x, p, "L")
        ZV, lpv = mix.phase(y, p, "V")
        lnK_new = lpl - lpv
        d = np.max(np.abs(lnK_new - lnK))
        lnK = lnK_new
        K = np.exp(lnK)
        if d < tol:
            converged = True
            break
        if np.max(np.abs(lnK)) < 1e-8:
            break
    two = (converged and beta is not None and 0.0 < beta < 1.0
           and np.max(np.abs(lnK)) > 1e-6)
    rhoL = p / (ZL * mix.RT)
    rhoV = p / (ZV * mix.RT)
    return FlashResult(beta if beta is not None else float("nan"), x, y, ZL, ZV,
                       rhoL, rhoV, it, converged, bool(two))


@dataclass
class Flash3Result:
    beta: np.ndarray      # phase mole fractions, in the order of the guesses
    x: np.ndarray         # [3][N] phase compositions
    Z: np.ndarray         # compressibility factor of each phase
    rho: np.ndarray       # molar density of each phase
    iterations: int
    converged: bool


def multiphase_rachford_rice(z, K, beta0, tol=1e-15, maxit=200):
    """Phase fractions of a multiphase split with K_ik = x_ik / x_i0 (phase 0
    the reference, K_i0 = 1): the zeros of
        h_k(beta) = sum_i z_i (K_ik - 1) / E_i,  E_i = 1 + sum_{k>0} beta_k (K_ik - 1),
    k > 0, i.e. sum_i x_ik = sum_i x_i0 (with x_ik = z_i K_ik / E_i).  Newton
    on the k > 0 fractions with the analytic Jacobian
        dh_k / dbeta_l = -sum_i z_i (K_ik - 1)(K_il - 1) / E_i^2,
    halving a step that would make some E_i non-positive."""
    z = np.asarray(z, dtype=np.float64)
    km1 = np.asarray(K, dtype=np.float64)[:, 1:] - 1.0          # [N][P-1]
    b = np.asarray(beta0, dtype=np.float64)[1:].copy()
    for _ in range(maxit):
        E = 1.0 + km1 @ b
        h = (z / E) @ km1
        J = -(km1 * (z / (E * E))[:, None]).T @ km1
        step = np.linalg.solve(J, -h)
        t = 1.0
        while np.any(1.0 + km1 @ (b + t * step) <= 0.0):
            t *= 0.5
        b = b + t * step
        if np.max(np.abs(t * step)) < tol:
            break
    return np.concatenate([[1.0 - b.sum()], b])


def flash3(mix, z, p, x0, labels, tol=1e-12, maxit=5000):
    """Isothermal three-phase flash at (T, p, z) by successive substitution
    on the K-values relative to phase 0 (the textbook multiphase extension
    of the two-phase flash above).

    x0: [3][N] initial compositions; labels: "V" or "L" per phase, which
    picks the largest or the smallest cubic root for that phase.  Each
    iteration: multiphase Rachford-Rice for the phase fractions, phase
    compositions from the mass balance, ln K_ik = ln phi_i0 - ln phi_ik.
    Stops when max |delta ln K| < tol.  At fixed T and p a three-component
    three-phase state has no free intensive variable (phase rule), so the
    compositions found do not depend on z inside the three-phase region."""
    z = np.asarray(z, dtype=np.float64)
    z = z / z.sum()
    x0 = np.asarray(x0, dtype=np.float64)
    lnK = np.log(x0 / x0[0])                 # [3][N]
    beta = np.full(3, 1.0 / 3.0)
    converged = False
    it = 0
    X = x0.copy()
    Z = np.zeros(3)
    for it in range(1, maxit + 1):
        K = np.exp(lnK).T                    # [N][3]
        beta = multiphase_rachford_rice(z, K, beta)
        E = K @ beta
        X = (z[:, None] * K / E[:, None]).T
        X = X / X.sum(axis=1, keepdims=True)
        lnphi = np.zeros((3, mix.N))
        for k in range(3):
            Z[k], lnphi[k] = mix.phase(X[k], p, labels[k])
        new = lnphi[0][None, :] - lnphi
        d = np.max(np.abs(new - lnK))
        lnK = new
        if d < tol:
            converged = True
            break
    rho = p / (Z * mix.RT)
    return Flash3Result(beta, X, Z.copy(), rho, it, converged)


def maxwell(mix, p0=None, tol=1e-14, maxit=200):
    """Saturation state of a pure component: equal pressure and fugacity.

    Newton on g(p) = ln phi_L(p) - ln phi_V(p) with dg/dp = (Z_L - Z_V) / p
    (the pressure derivative of ln phi at fixed T is (Z - 1)/p).  Returns
    (p_sat, rho_V, rho_L) in the mixture's units (molar densities).
    """
    assert mix.N == 1
    x = np.ones(1)
    p = float(wilson_K(mix, 1.0)[0]) if p0 is None else float(p0)
    lo, hi = 0.0, float(mix.pc[0])
    for _ in range(maxit):
        roots, _, _ = mix.z_roots(x, p)
        if len(roots) < 2 or roots[0] == roots[-1]:
            # outside the three-root band: bisect toward it
            Zs = roots[0] if roots else 1.0
            if Zs > 0.3:        # only a vapour-like root: pressure too low
                lo = p
            else:
                hi = p
            p = 0.5 * (lo + hi) if hi > lo else p * 0.9
            continue
        ZL, ZV = roots[0], roots[-1]
        g = float(mix.ln_phi(x, ZL, p)[0] - mix.ln_phi(x, ZV, p)[0])
        if g > 0.0:            # liquid less stable: below saturation
            lo = max(lo, p)
        else:
            hi = min(hi, p)
        dg = (ZL - ZV) / p
        pn = p - g / dg
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= tol * p:
            p = pn
            break
        p = pn
    roots, _, _ = mix.z_roots(x, p)
    ZL, ZV = roots[0], roots[-1]
    return p, p / (ZV * mix.RT), p / (ZL * mix.RT)


# ---------------------------------------------------------------------------
# Lattice units (Section III.A: R, a, b and M of the reference component are
# fixed; the same anchors recur in III.B, III.C and III.E)
# ---------------------------------------------------------------------------

class LatticeUnits:
    """Scales between SI and lattice units anchored on one component.

    With a_ref, b_ref and R fixed in lattice units, the reference component's
    critical temperature and pressure in lattice units follow from
    a = Omega_a R^2 Tc^2 / pc and b = Omega_b R Tc / pc.
    """

    def __init__(self, ref, a_lu=2.0 / 49.0, b_lu=2.0 / 21.0, R_lu=1.0, M_lu=1.0, eos="PR"):
        self.ref = ref
        self.eos = eos
        oa, ob = EOS[eos]["omega_a"], EOS[eos]["omega_b"]
        self.a_lu, self.b_lu, self.R_lu, self.M_lu = a_lu, b_lu, R_lu, M_lu
        self.Tc_ref_lu = (a_lu / b_lu) * (ob / oa) / R_lu
        self.pc_ref_lu = ob * R_lu * self.Tc_ref_lu / b_lu
        self.T_scale = ref.Tc / self.Tc_ref_lu                 # K per lu
        self.p_scale = ref.pc * BAR / self.pc_ref_lu            # Pa per lu
        b_ref_si = ob * R_SI * ref.Tc / (ref.pc * BAR)
        self.V_scale = b_ref_si / b_lu                          # m^3/mol per lu
        self.M_scale = ref.M / M_lu                             # g/mol per lu

    def T(self, T_K):
        return T_K / self.T_scale

    def p(self, p_Pa):
        return p_Pa / self.p_scale

    def rho_molar(self, rho_si):
        """mol/m^3 -> lattice molar density."""
        return np.asarray(rho_si) * self.V_scale

    def rho_molar_si(self, rho_lu):
        return np.asarray(rho_lu) / self.V_scale

    def mixture(self, comps, T_K, kij=None):
        """The PR mixture with every constant in lattice units."""
        Tc = np.array([c.Tc for c in comps]) / self.T_scale
        pc = np.array([c.pc * BAR for c in comps]) / self.p_scale
        om = np.array([c.omega for c in comps])
        return PRMixture(Tc, pc, om, self.T(T_K), kij, R=self.R_lu, eos=self.eos)

    def molar_masses(self, comps):
        return np.array([c.M for c in comps]) / self.M_scale


def si_mixture(comps, T_K, kij=None, eos="PR"):
    """The cubic-EOS mixture in SI units (Pa, m^3/mol)."""
    return PRMixture([c.Tc for c in comps], [c.pc * BAR for c in comps],
                     [c.omega for c in comps], T_K, kij, eos=eos)


def mass_density_si(comps, rho_molar_si_vec):
    """kg/m^3 of a phase from its component molar densities [mol/m^3]."""
    M = np.array([c.M for c in comps]) * 1e-3
    return float(np.dot(M, rho_molar_si_vec))
