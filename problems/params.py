"""Problem parameters: the same fields, names and enum values as ``grmhd_problem``."""

import math

NG = 3                      # ghost layers on each side of every direction

MINKOWSKI_CART, KERR_MKS, KERR_FMKS, KERR_CKS = 0, 1, 2, 3
RECON_MC, RECON_WENO5 = 0, 1
FP64, MIXED = 0, 1
BC_PERIODIC, BC_OUTFLOW, BC_POLAR, BC_DIRICHLET = 0, 1, 2, 3


def base_problem(n1, n2, n3, **kw):
    """Defaults for every ``grmhd_problem`` field.

    The floor constants are the bounds listed in the Implementation Notes
    section (rho > 1e-6 k, u > 1e-8 k^gamma, sigma < 400, beta > 2.5e-5,
    u/rho < 100, Lorentz factor < 50).
    """
    prm = dict(
        n1=int(n1), n2=int(n2), n3=int(n3),
        coords=MINKOWSKI_CART,
        a=0.0, gam=4.0 / 3.0, cfl=0.9,
        x1min=0.0, x1max=1.0, x2min=0.0, x2max=1.0, x3min=0.0, x3max=1.0,
        hslope=0.3, poly_xt=0.82, poly_alpha=14.0, mks_smooth=0.5,
        recon=RECON_MC, precision=FP64,
        bc=[[BC_PERIODIC, BC_PERIODIC], [BC_PERIODIC, BC_PERIODIC], [BC_PERIODIC, BC_PERIODIC]],
        floors=0,
        rho_fl=1e-6, u_fl=1e-8, sigma_max=400.0, beta_min=2.5e-5, uorho_max=100.0,
        gamma_max=50.0,
    )
    for k, v in kw.items():
        if k not in prm and not k.startswith("_"):
            raise KeyError(f"unknown problem field {k!r}")
        prm[k] = v
    return prm


def kerr_grid_extent(n1, a, r_out, zones_in_horizon=5.5):
    """Code-coordinate x1 extent of a Kerr grid (x1 = ln r).

    The outer edge sits at ln r_out; the inner edge is placed so that exactly
    ``zones_in_horizon`` zones lie inside the outer horizon r+ = 1 + sqrt(1-a^2).
    """
    rhor = 1.0 + math.sqrt(1.0 - a * a)
    x1max = math.log(r_out)
    x1min = (n1 * math.log(rhor) - zones_in_horizon * x1max) / (n1 - zones_in_horizon)
    return x1min, x1max


def padded_shape(prm, nvar=8):
    return (nvar, prm["n3"] + 2 * NG, prm["n2"] + 2 * NG, prm["n1"] + 2 * NG)
