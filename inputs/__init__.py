"""Seeded synthetic inputs shared by the GPU front end, the benchmark and the
CPU oracle's tests.

This package holds no step of the method: only component tables, initial
density profiles (the tanh profiles of the paper's Eq. (13) and (15), uniform
fields), seeded noise and parameter draws, and the phase states stored in
``phase_states.json`` (written offline by ``oracle/write_phase_states.py``).
"""
from .components import (Component, TABLE_I, TABLE_II, TABLE_V, DROPLET_3,  # noqa: F401
                          N_ALKANES, TERNARY_C1_C3_C10, table_ii_components)
from .fields import (droplet, slab, uniform, add_noise, draw_kij,  # noqa: F401
                     spinodal_z, load_phase_states)
