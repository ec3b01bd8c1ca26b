"""Plain, slow FP64 NumPy oracle of the per-zone GRMHD step.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it. It shares no code with the HIP library
(``paper_2110_10191_amd``), and the library does not import it.

What it computes is the HARM conservative finite-volume scheme for ideal GRMHD
that iharm3D implements (Functionality section), with Flux-CT (Implementation
Notes: Toth 2000), numerically evaluated metric quantities (Implementation
Notes), the 1D_W inversion (Implementation Notes: Noble et al. 2006) and the
bounds listed in the Implementation Notes. Where the paper defers to the HARM
literature the oracle writes the published method out; each such reading is
named in the docstring of the function that takes it.

Layout: primitives are float64 arrays ``[8, n3+6, n2+6, n1+6]`` (three ghost
layers per side, x1 fastest) in the order rho, u, u~1, u~2, u~3, B1, B2, B3.
Geometry of the axisymmetric coordinates (Minkowski, MKS, FMKS) is 2D tables
``[..., n2+6, n1+6]`` broadcast over x3; Cartesian Kerr-Schild, whose metric
depends on all three code coordinates, has 3D tables ``[..., n3+6, n2+6, n1+6]``
(``Grid.k3``), with its own x3-face table.

Electron heating (``oracle.electrons``): two advected entropies per zone and
the partition of the dissipated heat by a heating model; readings E1-E6 are
stated in that module, whose model formulas are parity unpinned beyond their
published limits.

Parity status per function (pins live in ``tests/test_oracle_*.py``):
every function is pinned to a closed form, an invariant or a brute-force
check, except the floor ordering and the fixup average, whose definitions are
readings of a silent passage (parity unpinned beyond idempotence, monotonicity
and order-independence).
"""

from .grid import Grid, NG
from .physics import fluid_state, flux, conserved, signal_speeds
from .recon import reconstruct, mc_slope, weno5_edge
from .invert import invert
from .step import (fill_ghosts, face_fluxes, flux_ct, substep, step, get_dt, divb,
                   prim_to_cons, cons_to_prim, run, floors, fixup, step_window)

__all__ = ["Grid", "NG", "fluid_state", "flux", "conserved", "signal_speeds",
           "reconstruct", "mc_slope", "weno5_edge", "invert", "fill_ghosts",
           "face_fluxes", "flux_ct", "substep", "step", "get_dt", "divb", "prim_to_cons",
           "cons_to_prim", "run", "floors", "fixup", "step_window"]
