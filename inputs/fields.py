"""Initial density fields and seeded draws (no thermodynamics here).

All fields are mass densities in lattice units, laid out [N][nz][ny][nx]
(C order), the layout the GPU library's ``fuglbm_init_fields`` takes.
"""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PHASE_STATES = os.path.join(HERE, "phase_states.json")


def droplet(nx, ny, rho_in, rho_out, R, W=4.0, centre=None):
    """Circular droplet, paper Eq. (13): liquid (``rho_in``) inside radius R."""
    rho_in = np.asarray(rho_in, dtype=np.float64)
    rho_out = np.asarray(rho_out, dtype=np.float64)
    xc, yc = (nx / 2.0, ny / 2.0) if centre is None else centre
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    r = np.sqrt((x - xc) ** 2 + (y - yc) ** 2)
    t = np.tanh(2.0 * (r - R) / W)
    out = (0.5 * (rho_in + rho_out))[:, None, None] - (0.5 * (rho_in - rho_out))[:, None, None] * t
    return out[:, None, :, :]


def slab(nx, ny, rho_V, rho_L, S_V, W=4.0, nz=1):
    """Flat liquid slab in the middle of a periodic box, paper Eq. (15)."""
    rho_V = np.asarray(rho_V, dtype=np.float64)
    rho_L = np.asarray(rho_L, dtype=np.float64)
    x = np.arange(nx, dtype=np.float64)
    prof = (np.tanh(2.0 * (x - 0.5 * S_V * nx) / W)
            - np.tanh(2.0 * (x - (1.0 - 0.5 * S_V) * nx) / W))
    out = rho_V[:, None] + 0.5 * (rho_L - rho_V)[:, None] * prof[None, :]
    return np.broadcast_to(out[:, None, None, :], (len(rho_V), nz, ny, nx)).copy()


def three_phase_slab(nx, ny, rho_V, rho_L1, rho_L2, W=8.0):
    """Eq. (16): liquid1 | vapour | liquid1 | liquid2 | liquid1 along x with
    tanh interfaces of width W at S1..S4 = nx/8, 3nx/8, 5nx/8, 7nx/8, one
    branch per quarter of the box.  The printed fourth branch names S1; the
    interface it describes sits at S4 (liquid2 -> liquid1 at 7nx/8)."""
    V, L1, L2 = (np.asarray(r, dtype=np.float64)[:, None] for r in (rho_V, rho_L1, rho_L2))
    x = np.arange(nx, dtype=np.float64)[None, :]

    def step(a, b, s):          # a for x << s, b for x >> s
        return 0.5 * (a + b) - 0.5 * (a - b) * np.tanh(2.0 * (x - s) / W)

    q = x <= nx / 4
    out = np.where(q, step(L1, V, nx / 8), 0.0)
    out = np.where((x > nx / 4) & (x <= nx / 2), step(V, L1, 3 * nx / 8), out)
    out = np.where((x > nx / 2) & (x <= 3 * nx / 4), step(L1, L2, 5 * nx / 8), out)
    out = np.where(x > 3 * nx / 4, step(L2, L1, 7 * nx / 8), out)
    return np.broadcast_to(out[:, None, None, :], (V.shape[0], 1, ny, nx)).copy()


def uniform(nx, ny, rho, nz=1):
    rho = np.asarray(rho, dtype=np.float64)
    return np.broadcast_to(rho[:, None, None, None], (len(rho), nz, ny, nx)).copy()


def add_noise(field, amplitude, seed):
    """rho <- rho (1 + A xi), xi ~ U[-1, 1) independent per component and site."""
    rng = np.random.Generator(np.random.PCG64(seed))
    xi = rng.uniform(-1.0, 1.0, size=field.shape)
    return field * (1.0 + amplitude * xi)


def draw_kij(n, lo, hi, seed):
    """Symmetric binary-interaction matrix with k_ii = 0, k_ij ~ U[lo, hi)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.zeros((n, n))
    iu = np.triu_indices(n, 1)
    k[iu] = rng.uniform(lo, hi, size=len(iu[0]))
    return k + k.T


def seeded_z(n, seed, concentration=20.0):
    """Overall composition drawn around equimolar: Dirichlet(concentration * 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.dirichlet(np.full(n, concentration))


def spinodal_z():
    """Overall composition of the ten-component n-alkane workload: the paper's
    Table VII composition with iC4+C4 and iC5+C5 merged and the CO2 and C7+
    fractions spread evenly over nC7..nC10."""
    z = np.array([0.6192, 0.1408, 0.0835, 0.0097 + 0.0341, 0.0084 + 0.0148, 0.0179,
                  0.0, 0.0, 0.0, 0.0])
    z[6:] = (0.0685 + 0.0031) / 4.0
    return z / z.sum()


def load_phase_states(path=PHASE_STATES):
    with open(path) as f:
        return json.load(f)
