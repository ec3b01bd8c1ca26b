"""Analytic pieces the Kerr initial data need: zone positions and the Kerr-Schild /
Boyer-Lindquist metrics at a point.

This is the grid *placement* only -- where each zone centre and corner sits in
(r, theta). The GRMHD step evaluates its own geometry independently.
"""

import math

import numpy as np

from .params import NG, KERR_MKS, KERR_FMKS


def theta_map(x1, x2, prm):
    """theta(x1, x2) and its partial derivatives for MKS / funky MKS.

    MKS:  theta_G = pi x2 + (1-h)/2 sin(2 pi x2).
    FMKS: y = 2 x2 - 1, theta_J = N y (1 + (y/xt)^alpha/(alpha+1)) + pi/2 with N
          chosen so theta_J(1) = pi; theta = theta_G + exp(-s (x1 - x1min)) (theta_J - theta_G).
    """
    h = prm["hslope"]
    thG = np.pi * x2 + 0.5 * (1.0 - h) * np.sin(2.0 * np.pi * x2)
    dthG = np.pi * (1.0 + (1.0 - h) * np.cos(2.0 * np.pi * x2))
    if prm["coords"] == KERR_MKS:
        return thG, np.zeros_like(thG + x1), dthG + 0.0 * x1
    assert prm["coords"] == KERR_FMKS
    xt, al, s = prm["poly_xt"], prm["poly_alpha"], prm["mks_smooth"]
    norm = 0.5 * np.pi / (1.0 + 1.0 / ((al + 1.0) * xt ** al))
    y = 2.0 * x2 - 1.0
    thJ = norm * y * (1.0 + (y / xt) ** al / (al + 1.0)) + 0.5 * np.pi
    dthJ = 2.0 * norm * (1.0 + (y / xt) ** al)
    e = np.exp(-s * (x1 - prm["x1min"]))
    th = thG + e * (thJ - thG)
    return th, -s * e * (thJ - thG), dthG + e * (dthJ - dthG)


def centres(prm, d, extra=NG):
    """Code coordinate of zone centres along direction d, ghosts included."""
    n = prm[f"n{d}"]
    lo, hi = prm[f"x{d}min"], prm[f"x{d}max"]
    dx = (hi - lo) / n
    return lo + (np.arange(-extra, n + extra) + 0.5) * dx, dx


def faces(prm, d, extra=NG):
    n = prm[f"n{d}"]
    lo, hi = prm[f"x{d}min"], prm[f"x{d}max"]
    dx = (hi - lo) / n
    return lo + np.arange(-extra, n + extra + 1) * dx, dx


def ks_gcov(r, th, a):
    """Kerr-Schild metric g_ab (t, r, theta, phi), shape [4, 4, ...]."""
    s2 = np.maximum(np.sin(th) ** 2, 1e-40)
    c2 = np.cos(th) ** 2
    sig = r * r + a * a * c2
    z = 2.0 * r / sig
    g = np.zeros((4, 4) + np.shape(r + th))
    g[0, 0] = -(1.0 - z)
    g[0, 1] = g[1, 0] = z
    g[0, 3] = g[3, 0] = -z * a * s2
    g[1, 1] = 1.0 + z
    g[1, 3] = g[3, 1] = -a * s2 * (1.0 + z)
    g[2, 2] = sig
    g[3, 3] = s2 * (sig + a * a * s2 * (1.0 + z))
    return g


def bl_quantities(r, th, a):
    """Boyer-Lindquist Sigma, Delta, A and the (t, phi) metric block."""
    s2 = np.sin(th) ** 2
    c2 = np.cos(th) ** 2
    sig = r * r + a * a * c2
    delta = r * r - 2.0 * r + a * a
    big_a = (r * r + a * a) ** 2 - delta * a * a * s2
    g_tt = -(1.0 - 2.0 * r / sig)
    g_tph = -2.0 * a * r * s2 / sig
    g_phph = big_a * s2 / sig
    return sig, delta, big_a, g_tt, g_tph, g_phph


def ks_to_code_velocity(vr, vth, vph, r, dth1, dth2):
    """Contravariant spatial KS components -> code components (t is unchanged).

    r = exp(x1), theta = theta(x1, x2), phi = x3, so
    v^1 = v^r / r,  v^2 = (v^theta - dtheta/dx1 v^1) / (dtheta/dx2),  v^3 = v^phi.
    """
    v1 = vr / r
    v2 = (vth - dth1 * v1) / dth2
    return v1, v2, vph


def normal_frame_velocity_ks(ut, ur, uth, uph, r, th, a):
    """u~^a = u^a - u^t g^{ta}/g^{tt} for a KS four-velocity.

    In Kerr-Schild g^{tt} = -(1 + 2r/Sigma), g^{tr} = 2r/Sigma and g^{t theta} =
    g^{t phi} = 0, so only the radial component picks up a shift.
    """
    sig = r * r + a * a * np.cos(th) ** 2
    return ur + ut * 2.0 * r / (sig + 2.0 * r), uth, uph


def horizon(a):
    return 1.0 + math.sqrt(1.0 - a * a)
