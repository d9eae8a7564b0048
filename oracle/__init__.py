"""CPU oracle of the fugacity-based multicomponent LBM (FP64).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py`` may import,
call or load anything in this package.  The GPU library
(``paper_2306_10652_amd``) never does, and the two share no code.

* ``thermo``     Peng-Robinson EOS (Eq. 9-12), lattice units, flash, Maxwell.
* ``lbm``        front of ``lbm_oracle.c``: the plain FP64 LBM step (Eq. 1-5).
* ``write_phase_states``  the only writer of the stored phase states
  (``inputs/phase_states.json``).

The bulk-window, Laplace-pressure and iso-fugacity read-outs of the
validation tests are written in those tests, over oracle thermodynamics.
"""
