"""Write ``inputs/phase_states.json``: the phase densities every synthetic
workload starts from, computed by the oracle's own flash / Maxwell code.

Run: ``python -m oracle.write_phase_states`` (from the repository root);
``python -m oracle.write_phase_states <group>`` (a key of ``PARTIAL``:
``vle_seeded``, ``droplet_c1c2c3``, ``ten_co2``, ``ternary_c1c2c3``, ``three_phase``)
refreshes only that group of states.
Only ``oracle/`` and the seeded draws in ``inputs/`` are used; nothing comes
from the GPU path.  All densities stored are lattice-unit MASS densities per
component (rho_i = M_i rho~_i), in the lattice units of each workload's own
anchor (its first component, a = 2/49, b = 2/21, R = 1, M = 1; the three-phase
case uses its own anchors, stored with it).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from inputs import components as C          # noqa: E402
from inputs import fields as Fi             # noqa: E402
from oracle import thermo as th             # noqa: E402
from oracle.lbm import oracle_mixture       # noqa: E402

BAR = th.BAR


def two_phase_state(comps, T, p_bar, z, kij=None):
    """Stability test and flash at (T, p, z) in lattice units; returns dict
    or None if one phase."""
    om = oracle_mixture(comps, T, kij)
    pr = om.pr
    p_lu = om.units.p(p_bar * BAR)
    if len(comps) == 1:
        ps, rV, rL = th.maxwell(pr)
        return dict(p_lu=ps, p_bar=ps * om.units.p_scale / BAR, beta=None, S_V=0.5,
                    rho_V=list(om.M * rV), rho_L=list(om.M * rL),
                    x=[1.0], y=[1.0])
    # Michelsen's stability test decides whether the feed splits; the flash
    # then gives the phases (a flash that finds no split of an unstable
    # feed, or a split of a stable one, rejects the draw)
    if th.stability(pr, z, p_lu).stable:
        return None
    r = th.flash(pr, z, p_lu)
    if not r.two_phase:
        return None
    vV, vL = 1.0 / r.rhoV, 1.0 / r.rhoL
    S_V = r.beta * vV / (r.beta * vV + (1.0 - r.beta) * vL)
    rho_V = om.M * r.y * r.rhoV
    rho_L = om.M * r.x * r.rhoL
    # overall (lever-rule) molar density of the two-phase state
    rho_tot = 1.0 / (r.beta * vV + (1.0 - r.beta) * vL)
    return dict(p_lu=p_lu, p_bar=p_bar, beta=r.beta, S_V=S_V,
                rho_V=list(rho_V), rho_L=list(rho_L), x=list(r.x), y=list(r.y),
                rho_uniform=list(om.M * np.asarray(z) / np.sum(z) * rho_tot))


def stable_in_oracle(comps, T, rho_V, rho_L, S_V, n, lattice=0, kij=None, steps=2000):
    """Screen a draw: the oracle advances a thin slab of the draw's own width
    (n x 2, or n x 2 x 2 for D3Q19) for `steps` steps without leaving the
    EOS domain.  High vapour/liquid density ratios with nearly absent heavy
    components make the scheme unstable at tau = 1; such draws are rejected."""
    from inputs import fields as Fi
    from oracle.lbm import OracleLBM
    m = oracle_mixture(comps, T, kij)
    nz = 2 if lattice == 1 else 1
    rho = Fi.slab(n, 2, rho_V, rho_L, S_V, nz=nz)
    o = OracleLBM(m, lattice, (n, 2, nz) if lattice == 1 else (n, 2), rho)
    for _ in range(steps // 250):
        if o.run(250) != 0:
            return False
    rr = o.rho()
    return bool(np.all(np.isfinite(rr)) and np.all(rr > 0))


def comp_list(comps):
    return [c._asdict() for c in comps]


def ternary_sweep(n_inst=256, seed=3):
    """Seeded two-phase draws for the batched ternary sweep (C1/C3/nC10)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    comps = C.TERNARY_C1_C3_C10
    out = []
    tries = 0
    while len(out) < n_inst and tries < 50000:
        tries += 1
        n = int(rng.integers(0, 13)) * 16 + 64          # 64..256 step 16
        T = float(rng.uniform(250.0, 450.0))
        p = float(rng.uniform(20.0, 150.0))
        z = rng.dirichlet(np.ones(3))
        st = two_phase_state(comps, T, p, z)
        if st is None or not (0.1 <= st["S_V"] <= 0.9):
            continue
        if np.max(np.abs(np.array(st["x"]) - np.array(st["y"]))) < 0.05:
            continue
        if not stable_in_oracle(comps, T, st["rho_V"], st["rho_L"], st["S_V"], n):
            continue
        st.update(n=n, T=T, p_bar_in=p, z=list(z))
        out.append(st)
    return out


def serving_pool(n_req=160, seed=5):
    """Seeded request pool for the serving stream (first N n-alkanes)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    tries = 0
    while len(out) < n_req and tries < 100000:
        tries += 1
        N = int(rng.integers(2, 11))
        three_d = bool(rng.uniform() < 0.2)
        n = int(rng.integers(0, 5)) * 16 + 64 if three_d else int(rng.integers(0, 29)) * 16 + 64
        T = float(rng.uniform(250.0, 450.0))
        p = float(rng.uniform(20.0, 150.0))
        z = rng.dirichlet(np.ones(N))
        comps = C.N_ALKANES[:N]
        st = two_phase_state(comps, T, p, z)
        if st is None or not (0.2 <= st["S_V"] <= 0.8):
            continue
        if np.max(np.abs(np.array(st["x"]) - np.array(st["y"]))) < 0.05:
            continue
        if not stable_in_oracle(comps, T, st["rho_V"], st["rho_L"], st["S_V"], n,
                                lattice=1 if three_d else 0):
            continue
        st.update(N=N, lattice="D3Q19" if three_d else "D2Q9", n=n, T=T, p_bar_in=p,
                  z=list(z), arrival_u=float(rng.uniform()))
        out.append(st)
    return out


def ten_co2_states():
    """Section III.E: the ten-component CO2 mixture at 150 bar; the flash at
    325 K (flat interface, Table VIII) and the uniform lever-rule densities
    at 325 K and 400 K (spinodal Cases 1 and 2, Tables IX-X)."""
    kij = np.array(C.ten_co2_kij())
    out = {}
    for T in (325.0, 400.0):
        st = two_phase_state(C.TEN_CO2, T, 150.0, C.TEN_CO2_Z, kij)
        st.update(components=comp_list(C.TEN_CO2), T=T, z=list(C.TEN_CO2_Z), kij=kij.tolist())
        out["ten_co2_%d" % int(T)] = st
    return out


def ternary_diagram_states(per_case=6, grid=12):
    """Section III.C: flat-interface states of the C1/C2/C3 ternary at the
    four (p, T) cases, over overall compositions on a simplex grid (step
    1/grid); per case the two-phase ones with 0.15 <= S_V <= 0.85 that the
    stability screen keeps, spread over the grid, at most per_case."""
    comps = C.TERNARY_C1_C2_C3
    out = []
    for case, (p, T) in sorted(C.TERNARY_CASES.items()):
        cand = []
        for a in range(1, grid):
            for b in range(1, grid - a):
                z = [a / grid, b / grid, (grid - a - b) / grid]
                st = two_phase_state(comps, T, p, z)
                if st is None or not (0.15 <= st["S_V"] <= 0.85):
                    continue
                cand.append((z, st))
        step = max(1, len(cand) // per_case)
        kept = 0
        for z, st in cand[::step]:
            if kept >= per_case:
                break
            if not stable_in_oracle(comps, T, st["rho_V"], st["rho_L"], st["S_V"], 400):
                continue
            st.update(case=case, T=T, p_bar_in=p, z=z)
            out.append(st)
            kept += 1
    return dict(components=comp_list(comps), instances=out)


def three_phase_state():
    """Section III.D: the C1/C4/CO2 three-phase flash at 225 K and 9 bar in
    the lattice units of the Table V anchors; phases in order vapour,
    liquid1, liquid2 (increasing mass density)."""
    comps = C.THREE_PHASE
    om = oracle_mixture(comps, C.THREE_PHASE_T_K, np.array(C.three_phase_kij()),
                        a_lu=C.THREE_PHASE_A_LU, b_lu=C.THREE_PHASE_B_LU)
    p_lu = om.units.p(C.THREE_PHASE_P_BAR * th.BAR)
    x0 = [[0.3, 0.02, 0.68], [0.01, 0.6, 0.39], [0.01, 0.1, 0.89]]
    r = th.flash3(om.pr, C.THREE_PHASE_Z, p_lu, x0, "VLL")
    assert r.converged
    S = r.beta / r.rho
    rho = [list(om.M * r.x[k] * r.rho[k]) for k in range(3)]
    return dict(components=comp_list(comps), T=C.THREE_PHASE_T_K,
                p_bar=C.THREE_PHASE_P_BAR, p_lu=p_lu, z=list(C.THREE_PHASE_Z),
                kij=C.three_phase_kij(), a_lu=C.THREE_PHASE_A_LU, b_lu=C.THREE_PHASE_B_LU,
                beta=list(r.beta), S=list(S / S.sum()), x=[list(v) for v in r.x],
                rho_V=rho[0], rho_L1=rho[1], rho_L2=rho[2])


def droplet_c1c2c3_state():
    """Section III.A: C1/C2/C3 (Table I, k_ij = 0) flashed at 250 K and 50 bar
    with z = (0.5, 0.25, 0.25), the droplet system of the Young-Laplace
    study."""
    comps = [C.TABLE_I["C1"], C.TABLE_I["C2"], C.TABLE_I["C3"]]
    st = two_phase_state(comps, 250.0, 50.0, [0.5, 0.25, 0.25])
    st.update(components=comp_list(comps), T=250.0)
    return st


def vle_seeded_states(seed=2):
    """Table II cases 2-6 at their (T, p) with the overall composition drawn
    around equimolar (Dirichlet(20 * 1), one draw per case from `seed`; a
    draw that does not split is replaced by the next)."""
    rng_seed = seed
    out = {}
    for case in range(2, 7):
        comps, T, p = C.table_ii_components(case)
        for k in range(100):
            z = Fi.seeded_z(len(comps), rng_seed * 100 + case * 10 + k)
            st = two_phase_state(comps, T, p, z)
            if st is not None and 0.2 <= st["S_V"] <= 0.8:
                break
        st.update(components=comp_list(comps), T=T, z=list(z), draw=k)
        out["vle%d_z2" % case] = st
    return out


PARTIAL = {"vle_seeded": lambda st: st.update(vle_seeded_states()),
           "droplet_c1c2c3": lambda st: st.update(droplet_c1c2c3=droplet_c1c2c3_state()),
           "ten_co2": lambda st: st.update(ten_co2_states()),
           "ternary_c1c2c3": lambda st: st.update(ternary_c1c2c3=ternary_diagram_states()),
           "three_phase": lambda st: st.update(three_phase=three_phase_state())}


def main(only=None):
    if only is not None:
        if only not in PARTIAL:
            raise SystemExit("unknown state group %r (known: %s)" % (only, ", ".join(PARTIAL)))
        with open(Fi.PHASE_STATES) as f:
            states = json.load(f)
        PARTIAL[only](states)
        with open(Fi.PHASE_STATES, "w") as f:
            json.dump(states, f, indent=1)
        print("updated", Fi.PHASE_STATES)
        return
    states = {}
    # 64x64 three-component droplet: 250 K, 50 bar, z = (0.5, 0.25, 0.25)
    st = two_phase_state(C.DROPLET_3, 250.0, 50.0, [0.5, 0.25, 0.25])
    st.update(components=comp_list(C.DROPLET_3), T=250.0, z=[0.5, 0.25, 0.25])
    states["droplet3"] = st
    # flat-interface VLE, Table II cases 1-6, equimolar z
    for case in range(1, 7):
        comps, T, p = C.table_ii_components(case)
        z = [1.0 / len(comps)] * len(comps)
        st = two_phase_state(comps, T, p, z)
        st.update(components=comp_list(comps), T=T, z=z)
        states["vle%d" % case] = st
    states.update(vle_seeded_states())
    # ten-component n-alkane spinodal: 325 K, 150 bar, seeded kij in [0, 0.05)
    kij = Fi.draw_kij(10, 0.0, 0.05, seed=4)
    z = Fi.spinodal_z()
    st = two_phase_state(C.N_ALKANES, 325.0, 150.0, z, kij)
    st.update(components=comp_list(C.N_ALKANES), T=325.0, z=list(z),
              kij=kij.tolist())
    states["spinodal10"] = st
    states["ternary_sweep"] = dict(components=comp_list(C.TERNARY_C1_C3_C10),
                                   instances=ternary_sweep())
    states["serving_pool"] = dict(components=comp_list(C.N_ALKANES),
                                  requests=serving_pool())
    states.update(ten_co2_states())
    states["ternary_c1c2c3"] = ternary_diagram_states()
    states["three_phase"] = three_phase_state()
    states["droplet_c1c2c3"] = droplet_c1c2c3_state()
    path = Fi.PHASE_STATES
    with open(path, "w") as f:
        json.dump(states, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    # a group name (see PARTIAL): add / refresh only that group
    main(sys.argv[1] if len(sys.argv) > 1 else None)
