"""MI355X-native hot path of the fugacity-based multicomponent lattice
Boltzmann method (per-step PR fugacity + interface force + well-balanced
collide-and-stream), fronted by the C ABI in ``include/fuglbm.h``.

* ``capi``     ctypes binding of ``libfuglbm.so`` (same names as the C ABI),
               ``Mixture`` / ``Simulation`` handle owners.
* ``batch``    batched sweeps (one launch per step for many simulations).
* ``serve``    continuous-batching simulation server.
* ``build``    in-tree hipcc build of the library for gfx950.
"""
