"""Pure-component property tables used to build synthetic workloads.

Data only: critical temperature Tc [K], critical pressure pc [bar], acentric
factor omega [-] and molar mass M [g/mol].  No thermodynamic arithmetic lives
here; both the CPU oracle and the GPU front end read these tables.
"""
from collections import namedtuple

Component = namedtuple("Component", "name Tc pc omega M")

# Paper, Section III, Table I (properties used in the LBM simulations).
TABLE_I = {
    "CO2": Component("CO2", 304.39, 73.843, 0.2667, 44.010),
    "C1": Component("C1", 190.74, 45.947, 0.0104, 16.043),
    "C2": Component("C2", 305.51, 48.711, 0.0979, 30.070),
    "C3": Component("C3", 370.03, 42.472, 0.1522, 44.097),
    "iC4": Component("iC4", 408.03, 36.397, 0.1852, 58.123),
    "C4": Component("C4", 425.34, 37.963, 0.1995, 58.123),
    "iC5": Component("iC5", 460.61, 33.812, 0.2280, 72.150),
    "C5": Component("C5", 469.89, 33.688, 0.2514, 72.150),
    "C6": Component("C6", 507.56, 30.123, 0.2994, 86.177),
    "C7+": Component("C7+", 617.78, 21.043, 0.4898, 142.285),
}

# Paper, Section III.D, Table V (three-phase case; slightly different values).
TABLE_V = {
    "CO2": Component("CO2", 304.20, 73.75, 0.2250, 44.010),
    "C1": Component("C1", 190.60, 45.99, 0.0080, 16.043),
    "C4": Component("C4", 425.20, 37.99, 0.1930, 58.123),
}

# Three-component droplet system of the 64x64 droplet workload (textbook
# critical constants; molar masses from Table I).
DROPLET_3 = [
    Component("C1", 190.6, 45.99, 0.011, 16.043),
    Component("C3", 369.8, 42.48, 0.152, 44.097),
    Component("nC5", 469.7, 33.70, 0.251, 72.150),
]

# n-alkane series C1..C10 for the ten-component spinodal workload.  C1-C6 are
# Table I rows (C4 = n-butane, C5 = n-pentane); nC7-nC9 are standard
# handbook critical constants (not in the paper); nC10 is the Table I "C7+"
# row, whose molar mass is that of n-decane.
N_ALKANES = [
    TABLE_I["C1"], TABLE_I["C2"], TABLE_I["C3"], TABLE_I["C4"], TABLE_I["C5"],
    TABLE_I["C6"],
    Component("nC7", 540.2, 27.40, 0.350, 100.204),
    Component("nC8", 568.7, 24.90, 0.399, 114.231),
    Component("nC9", 594.6, 22.90, 0.445, 128.258),
    Component("nC10", 617.78, 21.043, 0.4898, 142.285),
]

# Ternary used by the batched composition sweep: C1 / C3 / nC10.
TERNARY_C1_C3_C10 = [TABLE_I["C1"], TABLE_I["C3"], N_ALKANES[9]]

# Paper, Table II: components, temperature [K], pressure [bar] per case.
TABLE_II = {
    1: (["C1"], 177.24, 30.02),
    2: (["C1", "C2"], 215.00, 32.00),
    3: (["C1", "C2", "C3"], 250.00, 35.00),
    4: (["C1", "C2", "C3", "C4"], 300.00, 40.00),
    5: (["C1", "C2", "C3", "C4", "C5"], 350.00, 45.00),
    6: (["C1", "C2", "C3", "C4", "C5", "C6"], 400.00, 50.00),
}


def table_ii_components(case):
    names, T, p = TABLE_II[case]
    return [TABLE_I[n] for n in names], T, p


# Paper, Section III.E, Table VII: the ten-component mixture (Table I
# components) with its overall composition and the CO2 binary interaction
# parameters (all other pairs zero).  Ordered with C1 first, the component
# that anchors the lattice units (Section III.E fixes a, b and M of C1).
TEN_CO2_NAMES = ["C1", "C2", "C3", "iC4", "C4", "iC5", "C5", "C6", "C7+", "CO2"]
TEN_CO2 = [TABLE_I[n] for n in TEN_CO2_NAMES]
TEN_CO2_Z = [0.6192, 0.1408, 0.0835, 0.0097, 0.0341, 0.0084, 0.0148, 0.0179, 0.0685, 0.0031]
TEN_CO2_KIJ_CO2 = [0.105, 0.130, 0.125, 0.120, 0.115, 0.115, 0.115, 0.115, 0.115, 0.0]


def ten_co2_kij():
    """Symmetric k_ij matrix of the Table VII mixture (TEN_CO2 order)."""
    n = len(TEN_CO2)
    k = [[0.0] * n for _ in range(n)]
    c = TEN_CO2_NAMES.index("CO2")
    for i in range(n):
        k[i][c] = k[c][i] = TEN_CO2_KIJ_CO2[i]
    return k


# Paper, Section III.C: the C1/C2/C3 ternary (k_ij = 0) and its four
# pressure-temperature cases (bar, K).
TERNARY_C1_C2_C3 = [TABLE_I["C1"], TABLE_I["C2"], TABLE_I["C3"]]
TERNARY_CASES = {1: (45.0, 330.0), 2: (48.71, 305.51), 3: (50.0, 250.0), 4: (80.0, 275.0)}

# Paper, Section III.D: the three-phase C1/C4/CO2 case (Table V constants),
# k_ij(CO2, C1) = 0.12, k_ij(CO2, C4) = 0.15, the others zero; 225 K, 9 bar,
# z = (0.0194, 0.2643, 0.7163); lattice anchors R = 1, a_C1 = 0.011550,
# b_C1 = 0.107781, M_C1 = 1.
THREE_PHASE = [TABLE_V["C1"], TABLE_V["C4"], TABLE_V["CO2"]]
THREE_PHASE_Z = [0.0194, 0.2643, 0.7163]
THREE_PHASE_T_K = 225.0
THREE_PHASE_P_BAR = 9.0
THREE_PHASE_A_LU = 0.011550
THREE_PHASE_B_LU = 0.107781


def three_phase_kij():
    return [[0.0, 0.0, 0.12], [0.0, 0.0, 0.15], [0.12, 0.15, 0.0]]
