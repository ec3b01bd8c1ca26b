"""Electron heating (oracle): tracking dissipation and giving a share to the
electrons.

Implementation Notes: iharm3D can track dissipation and partition it between
ions and electrons (after Ressler et al. 2015), with five heating models
(Howes 2010, Kawazura et al. 2019, Werner et al. 2018, Rowan et al. 2017,
Sharma et al. 2007), and with electron temperatures evolved the bounds also
lower u until P_gas / rho^gamma < 3. The paper writes none of it out; the
readings taken here:

E1  two extra scalars per zone, the total entropy K_tot = P_gas / rho^gamma
    and the electron entropy K_e = P_e / rho^gamma_e (gamma_e = 4/3), held in
    a second padded array E = [K_tot, K_e] with the primitives' ghost rules
    for a scalar (periodic, copy, mirror without sign change, Dirichlet keep);
E2  both are advected with the mass flux: through a face the flux of rho u K
    is F_mass * K*, K* the reconstructed face value (the primitives'
    reconstruction) on the upwind side of F_mass (F_mass after Flux-CT, so the
    polar axis carries none);
E3  U_K = sqrt(-g) rho u^t K;  U_K(n+1) = U_K(base) - dt sum_d dF_K / dx_d,
    and K_adv = U_K(n+1) / (sqrt(-g) rho u^t) of the new, bounded, repaired
    primitives;
E4  after the other bounds, u <= kappa_max rho^gamma / (gamma - 1) with
    kappa_max = 3 (P_gas / rho^gamma < 3);
E5  the entropy the new internal energy implies, K = (gamma - 1) u / rho^gamma,
    exceeds the advected one by the dissipation; the electrons receive the
    fraction f_e of that heat:
      K_e <- K_e,adv + f_e (gamma_e - 1)/(gamma - 1) rho^(gamma - gamma_e) (K - K_tot,adv)
    bounded to [0, rho^(gamma - gamma_e) K] (P_e within [0, P_gas]), and
      K_tot <- K;
E6  f_e: a constant, or one of four models as functions of beta_i = P_i /
    (b^2/2), T_e/T_i = P_e / P_i (P_i = P_gas - P_e), sigma = b^2 / rho and
    sigma_w = b^2 / w (w = rho + u + P_gas):
      Kawazura 2019: Q_i/Q_e = 35 / (1 + (beta_i/15)^-1.4 exp(-0.1 T_e/T_i));
      Werner 2018:   f_e = (1 + sqrt((sigma/5) / (2 + sigma/5))) / 4;
      Rowan 2017:    f_e = exp(-(1 - beta_i/beta_max)^3.3 / (1 + 1.2 sigma_w^0.7)) / 2,
                     beta_max = 1/(4 sigma_w), (1 - beta_i/beta_max) floored at 0;
      Howes 2010:    with theta = T_i/T_e,
                     Q_i/Q_e = 0.92 (c2^2 + beta_i^x)/(c3^2 + beta_i^x) sqrt(m_p theta / m_e) exp(-1/beta_i),
                     x = 2 - 0.2 log10 theta; for theta > 1 c2 = 1.6/theta and
                     c3 = 18 + 5 log10 theta, for theta <= 1 c2 = 1.2/theta and
                     c3 = 18 (the two branches of that fit; beta_i^x capped at e^700);
      Sharma 2007:   Q_e/Q_i = sqrt(T_e/T_i) / 3, i.e. Q_i/Q_e = 3 sqrt(T_i/T_e)
                     (the electron-to-ion ratio that work fits; no formula in
                     the paper);
    with f_e = 1/(1 + Q_i/Q_e) where a ratio is given.

Parity status: E1-E5 are pinned by properties of the equations (a passive
scalar carried by a uniform flow converges to its exact translation at second
order; a uniform scalar stays uniform; ideal MHD is scale free, which fixes the
rho^(gamma - gamma_e) factor; electrons holding and receiving the same fraction
of entropy and heat keep it; the bounds hold). The model formulas of E6 are the
cited papers' as read here: parity unpinned beyond their published limits
(f_e -> 1 as beta_i -> 0 for Kawazura and Howes, Q_i/Q_e -> 35 at high beta_i
for Kawazura, Werner between 1/4 and 1/2, Rowan at most 1/2, Sharma 1/4 at
T_e = T_i). The Howes and Sharma coefficients in particular are read from the
cited works without a check against their tabulated values: parity unpinned.
"""

import numpy as np

from .grid import NG
from .physics import fluid_state
from .recon import reconstruct
from .step import (_interior, fill_ghosts, substep, dt_from_ctop, AXIS, BC_PERIODIC, BC_OUTFLOW,
                   BC_POLAR, BC_DIRICHLET)

GAM_E = 4.0 / 3.0
KAPPA_MAX = 3.0
MP_ME = 1836.15267343
MODEL_CONSTANT, MODEL_KAWAZURA, MODEL_WERNER, MODEL_ROWAN, MODEL_HOWES, MODEL_SHARMA = 0, 1, 2, 3, 4, 5


def fill_scalar_ghosts(E, grid, do_x3=True):
    """Ghost zones of a padded scalar array, in place (E1). With
    ``do_x3=False`` the x3 ghosts are real neighbour data of a window and are
    left alone."""
    prm = grid.prm
    n1, n2, n3 = grid.n
    bc = prm["bc"]
    K = slice(NG, NG + E.shape[1] - 2 * NG)
    J = slice(NG, NG + n2)
    for side in (0, 1):
        t = bc[0][side]
        for m in range(NG):
            g = NG - 1 - m if side == 0 else NG + n1 + m
            if t == BC_PERIODIC:
                s = NG + n1 - 1 - m if side == 0 else NG + m
            elif t == BC_OUTFLOW:
                s = NG if side == 0 else NG + n1 - 1
            else:
                continue
            E[:, K, J, g] = E[:, K, J, s]
    for side in (0, 1):
        t = bc[1][side]
        for m in range(NG):
            g = NG - 1 - m if side == 0 else NG + n2 + m
            if t == BC_PERIODIC:
                s = NG + n2 - 1 - m if side == 0 else NG + m
            elif t == BC_POLAR:
                s = NG + m if side == 0 else NG + n2 - 1 - m
            elif t == BC_OUTFLOW:
                s = NG if side == 0 else NG + n2 - 1
            else:
                continue
            E[:, K, g, :] = E[:, K, s, :]
    for side in (0, 1):
        t = bc[2][side] if do_x3 else BC_DIRICHLET
        for m in range(NG):
            g = NG - 1 - m if side == 0 else NG + n3 + m
            if t == BC_PERIODIC:
                s = NG + n3 - 1 - m if side == 0 else NG + m
            elif t == BC_OUTFLOW:
                s = NG if side == 0 else NG + n3 - 1
            else:
                continue
            E[:, g, :, :] = E[:, s, :, :]
    return E


def scalar_fluxes(E, mass, grid, d):
    """F_K at the lower d-faces (E2): mass flux times the upwind face value."""
    ax = AXIS[d]
    n = E.shape[ax] - 2 * NG
    f0, f1 = NG, NG + n + 1
    KL, KR = reconstruct(E, ax, grid.prm["recon"], f0, f1)
    sl = [slice(None)] * 3
    sl[ax - 1] = slice(f0, f1)
    m = mass[tuple(sl)]
    Fk = np.full(E.shape, np.nan)
    Fk[(slice(None),) + tuple(sl)] = m * np.where(m >= 0.0, KL, KR)
    return Fk


def heating_fraction(model, fel, rho, u, kel, bsq, gam):
    """f_e of E6 at each zone."""
    if model == MODEL_CONSTANT:
        return np.full(np.shape(rho), float(fel))
    pg = (gam - 1.0) * u
    pe = kel * rho ** GAM_E
    pi = np.maximum(pg - pe, 1e-30 * pg + 1e-300)
    pb = 0.5 * bsq + 1e-300
    beta = pi / pb
    te_ti = pe / pi
    if model == MODEL_KAWAZURA:
        qi_qe = 35.0 / (1.0 + (beta / 15.0) ** -1.4 * np.exp(-0.1 * te_ti))
        return 1.0 / (1.0 + qi_qe)
    if model == MODEL_WERNER:
        s5 = bsq / rho / 5.0
        return 0.25 * (1.0 + np.sqrt(s5 / (2.0 + s5)))
    if model == MODEL_ROWAN:
        sw = bsq / (rho + u + pg)
        bmax = 1.0 / (4.0 * sw + 1e-300)
        x = np.maximum(1.0 - beta / bmax, 0.0)
        return 0.5 * np.exp(-x ** 3.3 / (1.0 + 1.2 * sw ** 0.7))
    if model == MODEL_HOWES:
        theta = pi / np.maximum(pe, 1e-300)
        lt = np.log10(theta)
        c2 = np.where(theta > 1.0, 1.6, 1.2) / theta
        c3 = np.where(theta > 1.0, 18.0 + 5.0 * lt, 18.0)
        x = 2.0 - 0.2 * lt
        bx = np.exp(np.minimum(x * np.log(beta), 700.0))   # beta^x, kept finite
        qi_qe = 0.92 * (c2 * c2 + bx) / (c3 * c3 + bx) * np.sqrt(MP_ME * theta) * np.exp(-1.0 / beta)
        return 1.0 / (1.0 + qi_qe)
    if model == MODEL_SHARMA:
        qi_qe = 3.0 * np.sqrt(pi / np.maximum(pe, 1e-300))
        return 1.0 / (1.0 + qi_qe)
    raise ValueError(f"unknown heating model {model}")


def electron_substep(Es, Eb, Pb, Pn, mass, grid, dt, model, fel):
    """E after one substep (E3-E5). Es: flux-state scalars, ghosts filled
    (padded); Eb, Pb: base state on the interior; Pn: the substep's new,
    bounded, repaired primitives on the interior (its u is lowered in place by
    E4). Returns the new scalars on the interior."""
    prm = grid.prm
    gam = prm["gam"]
    n1, n2 = grid.n[0], grid.n[1]
    n3 = Pn.shape[1]                # the block's x3 extent (a window of the domain, or all of it)
    K, J, I = slice(NG, NG + n3), slice(NG, NG + n2), slice(NG, NG + n1)
    Kp, Jp, Ip = slice(NG + 1, NG + n3 + 1), slice(NG + 1, NG + n2 + 1), slice(NG + 1, NG + n1 + 1)
    F1 = scalar_fluxes(Es, mass[0], grid, 1)
    F2 = scalar_fluxes(Es, mass[1], grid, 2)
    F3 = scalar_fluxes(Es, mass[2], grid, 3)
    dx1, dx2, dx3 = grid.dx
    div = ((F1[:, K, J, Ip] - F1[:, K, J, I]) / dx1 + (F2[:, K, Jp, I] - F2[:, K, J, I]) / dx2
           + (F3[:, Kp, J, I] - F3[:, K, J, I]) / dx3)
    geo = grid.sub(grid.cent, K, J, I)
    gdet = geo["gdet"]
    sb = fluid_state(Pb, geo, gam)
    Ub = gdet * Pb[0] * sb["ucon"][0] * Eb
    Uk = Ub - dt * div
    # E4 on the new state, then its implied entropy
    rho = Pn[0]
    Pn[1] = np.minimum(Pn[1], KAPPA_MAX * rho ** gam / (gam - 1.0))
    sn = fluid_state(Pn, geo, gam)
    dn = gdet * rho * sn["ucon"][0]
    kadv = Uk / dn
    ktot = (gam - 1.0) * Pn[1] / rho ** gam
    fe = heating_fraction(model, fel, rho, Pn[1], kadv[1], sn["bsq"], gam)
    scale = rho ** (gam - GAM_E)
    kel = kadv[1] + fe * (GAM_E - 1.0) / (gam - 1.0) * scale * (ktot - kadv[0])
    kel = np.minimum(np.maximum(kel, 0.0), scale * ktot)
    return np.array([ktot, kel])


def step(P, E, grid, dt, model=MODEL_CONSTANT, fel=0.5):
    """One predictor-corrector step of primitives and electron scalars.
    Returns (P_new, E_new, dt_next)."""
    n1, n2, n3 = grid.n
    it = _interior(n3, n2, n1)
    P0 = fill_ghosts(P.copy(), grid)
    E0 = fill_scalar_ghosts(E.copy(), grid)
    Ph_i, _, _, m1 = substep(P0, P0[it], grid, 0.5 * dt, mass_flux=True)
    Eh_i = electron_substep(E0, E0[it], P0[it], Ph_i, m1, grid, 0.5 * dt, model, fel)
    Ph = P0.copy()
    Ph[it] = Ph_i
    Eh = E0.copy()
    Eh[it] = Eh_i
    fill_ghosts(Ph, grid)
    fill_scalar_ghosts(Eh, grid)
    Pn_i, _, cmax, m2 = substep(Ph, P0[it], grid, dt, mass_flux=True)
    En_i = electron_substep(Eh, E0[it], P0[it], Pn_i, m2, grid, dt, model, fel)
    Pn = P0.copy()
    Pn[it] = Pn_i
    En = E0.copy()
    En[it] = En_i
    return Pn, En, dt_from_ctop(cmax, grid)



def step_window(P, E, grid, dt, k0, k1, model=MODEL_CONSTANT, fel=0.5):
    """(P^{n+1}, E^{n+1}) on interior slabs k0..k1-1 of full padded states,
    computed from a window of x3 slabs around them, as the fluid window step
    does (the scalars need no wider margin than the fluid: their face values
    use the same stencil and their fluxes the fluid's mass fluxes)."""
    n1, n2, n3 = grid.n
    full = fill_ghosts(P.copy(), grid)
    fullE = fill_scalar_ghosts(E.copy(), grid)
    M1 = 5
    ks = np.arange(k0 - M1 - NG, k1 + M1 + NG) % n3 + NG
    blk, eblk = full[:, ks], fullE[:, ks]
    it1 = (slice(None), slice(NG, blk.shape[1] - NG), slice(NG, NG + n2), slice(NG, NG + n1))
    Ph_i, _, _, m1 = substep(blk, blk[it1], grid, 0.5 * dt, mass_flux=True, window=True)
    Eh_i = electron_substep(eblk, eblk[it1], blk[it1], Ph_i, m1, grid, 0.5 * dt, model, fel)
    ph, eh = blk.copy(), eblk.copy()
    ph[it1], eh[it1] = Ph_i, Eh_i
    fill_ghosts(ph, grid, do_x3=False)
    fill_scalar_ghosts(eh, grid, do_x3=False)
    off = (M1 + NG) - (1 + NG)
    w = (k1 - k0) + 2 + 2 * NG
    blk2, eblk2 = ph[:, off:off + w], eh[:, off:off + w]
    inner = (slice(None), slice(off + NG, off + NG + (k1 - k0) + 2), slice(NG, NG + n2), slice(NG, NG + n1))
    Pn_i, _, _, m2 = substep(blk2, blk[inner], grid, dt, mass_flux=True, window=True)
    En_i = electron_substep(eblk2, eblk[inner], blk[inner], Pn_i, m2, grid, dt, model, fel)
    return Pn_i[:, 1:-1], En_i[:, 1:-1]
