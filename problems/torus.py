"""Fishbone-Moncrief torus in Kerr, on a funky-MKS grid (or plain MKS with
``coords=KERR_MKS``).

The accretion-torus problem of the Scaling section. Units GM = c = 1 and the
density normalised to a maximum of 1 (Implementation Notes section).

Construction (Fishbone & Moncrief 1976; Bardeen, Press & Teukolsky 1972):

* specific angular momentum l = u^t u_phi of the prograde circular orbit at r_max;
* enthalpy ln h(r, theta) relative to the inner edge (r_in, pi/2); inside the torus
  rho ~ (h-1)^(1/(gamma-1)) and u = rho (h-1)/gamma;
* circular Boyer-Lindquist velocity, which Kerr-Schild leaves unchanged (u^r = 0);
* single-loop field from A_phi = max(<rho> - 0.2, 0) at zone corners, scaled to
  max p_gas / max p_mag = beta;
* seeded uniform multiplicative noise on u; atmosphere rho = rho_fl k, u = u_fl k^gamma,
  u~ = 0, with k = 1/(r^2 (1 + r/10)).
"""

import math

import numpy as np

from .params import (NG, KERR_FMKS, RECON_MC, FP64, BC_OUTFLOW, BC_POLAR, BC_PERIODIC,
                     base_problem, kerr_grid_extent)
from .kerr import (theta_map, centres, ks_gcov, bl_quantities, ks_to_code_velocity,
                   normal_frame_velocity_ks)


def circular_orbit_ell(r, a):
    """u^t u_phi of the prograde equatorial circular orbit at radius r (BPT 1972)."""
    den = r ** 0.75 * math.sqrt(r ** 1.5 - 3.0 * math.sqrt(r) + 2.0 * a)
    ut = (r ** 1.5 + a) / den
    uph = (r * r - 2.0 * a * math.sqrt(r) + a * a) / den
    return ut * uph


def fm_lnh(r, th, a, ell, rin):
    """ln h(r, theta) - ln h(r_in, pi/2) for the constant-l torus (NaN or inf
    where the expression has no real value, e.g. inside the horizon or on the
    axis; callers keep only the torus body, where ln h > 0)."""
    def raw(r, th):
        sig, delta, big_a, _, _, _ = bl_quantities(r, th, a)
        s2 = np.sin(th) ** 2
        with np.errstate(invalid="ignore", divide="ignore"):
            q = np.sqrt(1.0 + 4.0 * ell * ell * sig * sig * delta / (big_a * big_a * s2))
            return 0.5 * np.log((1.0 + q) / (sig * delta / big_a)) - 0.5 * q - 2.0 * a * r * ell / big_a
    return raw(r, th) - raw(np.float64(rin), np.float64(0.5 * np.pi))


def fm_torus(n1=288, n2=128, n3=128, a=0.9375, rin=6.0, rmax=12.0, gam=13.0 / 9.0,
             r_out=1000.0, beta=100.0, seed=2, noise=0.04, recon=RECON_MC, precision=FP64,
             coords=KERR_FMKS, hslope=0.3):
    x1min, x1max = kerr_grid_extent(n1, a, r_out)
    prm = base_problem(
        n1, n2, n3, coords=coords, a=a, gam=gam, hslope=hslope,
        x1min=x1min, x1max=x1max, x2min=0.0, x2max=1.0, x3min=0.0, x3max=2.0 * math.pi,
        bc=[[BC_OUTFLOW, BC_OUTFLOW], [BC_POLAR, BC_POLAR], [BC_PERIODIC, BC_PERIODIC]],
        floors=1, recon=recon, precision=precision,
        _name="fm_torus", _seed=seed, _rin=rin, _rmax=rmax, _beta=beta, _noise=noise)

    x1c, dx1 = centres(prm, 1)
    x2c, dx2 = centres(prm, 2)
    X1, X2 = np.meshgrid(x1c, x2c)                 # [J, I] padded
    th, dth1, dth2 = theta_map(X1, X2, prm)
    r = np.exp(X1)
    ell = circular_orbit_ell(rmax, a)

    # torus body (evaluated at ghost centres too: the corner potential needs them)
    lnh = np.full_like(r, -1.0)
    ok = r >= rin
    with np.errstate(invalid="ignore", divide="ignore"):
        lnh[ok] = fm_lnh(r[ok], th[ok], a, ell, rin)
    inside = ok & (lnh > 0.0)
    hm1 = np.where(inside, np.expm1(np.where(inside, lnh, 0.0)), 0.0)
    rho_t = np.where(inside, hm1 ** (1.0 / (gam - 1.0)), 0.0)
    u_t = rho_t * hm1 / gam

    sl = (slice(NG, NG + n2), slice(NG, NG + n1))
    rhomax = rho_t[sl].max()
    rho_t /= rhomax
    u_t /= rhomax

    # circular velocity in Boyer-Lindquist, then normal-frame KS, then code components
    with np.errstate(invalid="ignore", divide="ignore"):
        sig, delta, big_a, g_tt, g_tph, g_phph = bl_quantities(r, th, a)
        s2 = np.sin(th) ** 2
        x = (g_phph + np.sqrt(g_phph ** 2 + 4.0 * ell * ell * delta * s2)) / (2.0 * delta * s2)
        ut = np.sqrt(x)
        uph = (ell - g_tph * x) / (g_phph * ut)
    ut = np.where(inside, ut, 0.0)
    uph = np.where(inside, uph, 0.0)
    vr, vth, vph = normal_frame_velocity_ks(ut, 0.0 * ut, 0.0 * ut, uph, r, th, a)
    v1, v2, v3 = ks_to_code_velocity(vr, vth, vph, r, dth1, dth2)

    kfl = 1.0 / (r * r * (1.0 + r / 10.0))
    rho = np.where(inside, rho_t, prm["rho_fl"] * kfl)
    uu = np.where(inside, u_t, prm["u_fl"] * kfl ** gam)

    # single-loop field: A_phi at corner (i-1/2, j-1/2) from the 4 adjacent centres
    rb = 0.25 * (rho_t[:-1, :-1] + rho_t[1:, :-1] + rho_t[:-1, 1:] + rho_t[1:, 1:])
    A = np.maximum(rb - 0.2, 0.0)                  # A[jc, ic]: corner below/left of padded zone (jc+1, ic+1)
    # corners of interior zone (j, i) sit at padded corner indices NG-1+j .. NG+j (same for i)
    Aj0 = A[NG - 1:NG - 1 + n2, :]
    Aj1 = A[NG:NG + n2, :]
    A00 = Aj0[:, NG - 1:NG - 1 + n1]; A10 = Aj0[:, NG:NG + n1]
    A01 = Aj1[:, NG - 1:NG - 1 + n1]; A11 = Aj1[:, NG:NG + n1]
    gdet = (sig * np.abs(np.sin(th)) * r * dth2)[sl]
    B1 = -(A00 - A01 + A10 - A11) / (2.0 * dx2 * gdet)
    B2 = (A00 + A01 - A10 - A11) / (2.0 * dx1 * gdet)

    # normalise to max p_gas / max p_mag = beta, with b^2 evaluated in Kerr-Schild
    ri, thi = r[sl], th[sl]
    g = ks_gcov(ri, thi, a)
    br, bth = ri * B1, dth1[sl] * B1 + dth2[sl] * B2
    Bks = np.array([np.zeros_like(br), br, bth, np.zeros_like(br)])
    vks = np.array([np.zeros_like(br), vr[sl], vth[sl] + 0.0 * br, vph[sl]])
    gam_n = np.sqrt(1.0 + np.einsum("ij...,i...,j...->...", g[1:, 1:], vks[1:], vks[1:]))
    sigi = ri * ri + a * a * np.cos(thi) ** 2
    alpha = 1.0 / np.sqrt(1.0 + 2.0 * ri / sigi)
    ucon = np.array([gam_n / alpha, vks[1] - gam_n * alpha * 2.0 * ri / sigi, vks[2], vks[3]])
    ucov = np.einsum("ab...,b...->a...", g, ucon)
    bdotu = np.einsum("i...,i...->...", Bks[1:], ucov[1:])
    bsq = (np.einsum("ij...,i...,j...->...", g[1:, 1:], Bks[1:], Bks[1:]) + bdotu ** 2) / ucon[0] ** 2
    pgas = (gam - 1.0) * uu[sl]
    beta_act = pgas.max() / (0.5 * bsq).max()
    f = math.sqrt(beta_act / beta)
    B1 *= f
    B2 *= f
    prm["_beta_before_scaling"] = float(beta_act)

    P = np.zeros((8, n3 + 2 * NG, n2 + 2 * NG, n1 + 2 * NG))
    isl = (slice(NG, NG + n3),) + sl
    P[0][isl] = rho[sl]
    P[1][isl] = uu[sl]
    P[2][isl] = v1[sl]
    P[3][isl] = v2[sl]
    P[4][isl] = v3[sl]
    P[5][isl] = B1
    P[6][isl] = B2

    rng = np.random.default_rng(seed)
    xi = rng.random((n3, n2, n1))
    P[1][isl] *= np.where(inside[sl], 1.0 + noise * (xi - 0.5), 1.0)
    return prm, P
