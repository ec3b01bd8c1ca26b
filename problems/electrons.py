"""Initial electron-heating entropies of a problem (input generation only)."""

import numpy as np

GAM_E = 4.0 / 3.0


def electron_scalars(P, gam, te_ti=1.0):
    """[2, ...] padded array of K_tot = P_gas / rho^gam and K_e = P_e / rho^(4/3)
    for electrons at T_e/T_i = te_ti (P_e = P_gas te_ti / (1 + te_ti)); zones
    with rho <= 0 (unset ghosts) are taken at rho = 1."""
    rho = np.where(P[0] > 0, P[0], 1.0)
    pg = (gam - 1.0) * P[1]
    ktot = pg / rho ** gam
    kel = pg * te_ti / (1.0 + te_ti) / rho ** GAM_E
    return np.array([ktot, kel])
