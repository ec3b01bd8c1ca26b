"""Seeded synthetic initial data for the workloads of the method.

The test problems are the ones the paper evolves (Tests and Scaling sections):
linear MHD modes on a periodic 3D box, un-magnetised Bondi accretion, and the
Fishbone-Moncrief accretion torus; plus magnetised spherical accretion on a
Cartesian Kerr-Schild box, a spacetime whose geometry depends on x3. This package only *places analytic
solutions on the grid*: it holds none of the step's arithmetic (no fluxes,
reconstruction, inversion or floors). Both the HIP library and the CPU oracle
receive its output as input.

Every generator returns ``(prm, P)``:

* ``prm`` -- a plain dict whose keys are exactly the fields of the C struct
  ``grmhd_problem`` (see ``include/grmhd.h``), plus a few bookkeeping keys
  prefixed with ``_``;
* ``P`` -- float64 primitives ``[8, n3+6, n2+6, n1+6]`` (3 ghost layers on each
  side, x1 fastest). Interior zones hold the initial data; ghost zones hold
  the analytic solution where a boundary is Dirichlet and zeros elsewhere.

Primitive order: rho, u (internal energy density), u~1, u~2, u~3 (velocity
relative to the normal observer, code coordinates), B1, B2, B3.
"""

from .params import (NG, MINKOWSKI_CART, KERR_MKS, KERR_FMKS, KERR_CKS, RECON_MC, RECON_WENO5,
                     FP64, MIXED, BC_PERIODIC, BC_OUTFLOW, BC_POLAR, BC_DIRICHLET,
                     base_problem, kerr_grid_extent, padded_shape)
from .modes import linear_modes, mode_solution
from .torus import fm_torus
from .bondi import bondi
from .cks import cks_bondi
from .electrons import electron_scalars

__all__ = [
    "NG", "MINKOWSKI_CART", "KERR_MKS", "KERR_FMKS", "KERR_CKS", "RECON_MC", "RECON_WENO5",
    "FP64", "MIXED", "BC_PERIODIC", "BC_OUTFLOW", "BC_POLAR", "BC_DIRICHLET",
    "base_problem", "kerr_grid_extent", "padded_shape",
    "linear_modes", "mode_solution", "fm_torus", "bondi", "cks_bondi", "electron_scalars",
]
