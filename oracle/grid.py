"""Coordinates, metric and connection (oracle).

Implementation Notes section: every metric-dependent quantity is evaluated
numerically from the line element in analytic form, and the coordinates act
as static mesh refinement. Here:

* Minkowski: Cartesian code coordinates, g = diag(-1, 1, 1, 1).
* Kerr: Kerr-Schild (t, r, theta, phi) with code coordinates r = exp(x1),
  theta = theta(x1, x2) (MKS, or "funky" MKS which blends in a polynomial
  theta_J(x2) that flattens the resolution near the poles), phi = x3.
  g_code = J^T g_KS J with the analytic Jacobian J = d(t,r,theta,phi)/d(x0..x3).
* g^{mu nu} is the numerical inverse, sqrt(-g) the square root of minus the
  numerical determinant, alpha = 1/sqrt(-g^{tt}).
* The connection Gamma^l_{mn} = g^{lk} Gamma_{kmn}, Gamma_{kmn} =
  (d_n g_km + d_m g_kn - d_k g_mn)/2, with the derivatives taken by centred
  differences of g_code in x1 and x2 (step 1e-5); d_t = d_x3 = 0.

Reading (the paper gives no formula for the coordinates): the MKS/FMKS maps of
the HARM literature, with h = 0.3, x_t = 0.82, alpha = 14, s = 0.5; |sin theta|
is kept >= 1e-20 inside the metric so that faces on the polar axis keep an
invertible metric.
"""

import numpy as np

NG = 3
MINKOWSKI_CART, KERR_MKS, KERR_FMKS = 0, 1, 2
FD_DELTA = 1e-5
SIN_MIN = 1e-20


def theta_of(x1, x2, prm):
    """theta and its partial derivatives d theta/dx1, d theta/dx2."""
    h = prm["hslope"]
    tg = np.pi * x2 + 0.5 * (1.0 - h) * np.sin(2.0 * np.pi * x2)
    dtg = np.pi + np.pi * (1.0 - h) * np.cos(2.0 * np.pi * x2)
    if prm["coords"] == KERR_MKS:
        return tg + 0.0 * x1, 0.0 * (x1 + x2), dtg + 0.0 * x1
    xt = prm["poly_xt"]
    al = prm["poly_alpha"]
    s = prm["mks_smooth"]
    norm = (np.pi / 2.0) / (1.0 + 1.0 / ((al + 1.0) * xt ** al))
    y = 2.0 * x2 - 1.0
    tj = norm * y * (1.0 + (y / xt) ** al / (al + 1.0)) + np.pi / 2.0
    dtj = 2.0 * norm * (1.0 + (y / xt) ** al)
    blend = np.exp(-s * (x1 - prm["x1min"]))
    th = tg + blend * (tj - tg)
    return th, -s * blend * (tj - tg), dtg + blend * (dtj - dtg)


def gcov_ks(r, th, a):
    """Kerr metric in Kerr-Schild coordinates, [4, 4, ...]."""
    sth = np.sin(th)
    sth = np.where(np.abs(sth) < SIN_MIN, SIN_MIN, sth)
    s2 = sth * sth
    c2 = np.cos(th) ** 2
    rho2 = r * r + a * a * c2
    f = 2.0 * r / rho2
    out = np.zeros((4, 4) + np.shape(r * th), dtype=np.result_type(r, th, 1.0))
    out[0, 0] = -(1.0 - f)
    out[0, 1] = out[1, 0] = f
    out[0, 3] = out[3, 0] = -a * f * s2
    out[1, 1] = 1.0 + f
    out[1, 3] = out[3, 1] = -a * s2 * (1.0 + f)
    out[2, 2] = rho2
    out[3, 3] = s2 * (rho2 + a * a * s2 * (1.0 + f))
    return out


def gcov_code(x1, x2, prm):
    """Covariant metric in code coordinates at (x1, x2), [4, 4, ...]."""
    shape = np.shape(x1 + x2)
    if prm["coords"] == MINKOWSKI_CART:
        g = np.zeros((4, 4) + shape)
        g[0, 0] = -1.0
        g[1, 1] = g[2, 2] = g[3, 3] = 1.0
        return g
    r = np.exp(x1)
    th, dth1, dth2 = theta_of(x1, x2, prm)
    gks = gcov_ks(r, th, prm["a"])
    J = np.zeros((4, 4) + shape, dtype=np.result_type(x1, x2, 1.0))  # J[a, mu] = d x_KS^a / d X^mu
    J[0, 0] = 1.0
    J[1, 1] = r
    J[2, 1] = dth1
    J[2, 2] = dth2
    J[3, 3] = 1.0
    g = np.einsum("am...,ab...,bn...->mn...", J, gks, J)
    for m in range(4):                    # exactly symmetric
        for n in range(m + 1, 4):
            g[n, m] = g[m, n]
    return g


def metric(x1, x2, prm):
    """dict(gcov, gcon, gdet, alpha) at (x1, x2)."""
    g = gcov_code(x1, x2, prm)
    gm = np.moveaxis(g, (0, 1), (-2, -1))
    gcon = np.moveaxis(np.linalg.inv(gm), (-2, -1), (0, 1))
    gdet = np.sqrt(np.abs(np.linalg.det(gm)))
    alpha = 1.0 / np.sqrt(-gcon[0, 0])
    return dict(gcov=g, gcon=gcon, gdet=gdet, alpha=alpha)


def connection(x1, x2, prm, delta=FD_DELTA):
    """Gamma^l_{mn}, [4, 4, 4, ...], from centred differences of g_code."""
    shape = np.shape(x1 + x2)
    dg = np.zeros((4, 4, 4) + shape)      # dg[c, a, b] = d_c g_ab
    if prm["coords"] != MINKOWSKI_CART:
        dg[1] = (gcov_code(x1 + delta, x2, prm) - gcov_code(x1 - delta, x2, prm)) / (2.0 * delta)
        dg[2] = (gcov_code(x1, x2 + delta, prm) - gcov_code(x1, x2 - delta, prm)) / (2.0 * delta)
    # Gamma_{k m n} = (d_n g_km + d_m g_kn - d_k g_mn) / 2
    low = 0.5 * (np.einsum("nkm...->kmn...", dg) + np.einsum("mkn...->kmn...", dg)
                 - np.einsum("kmn...->kmn...", dg))
    gcon = metric(x1, x2, prm)["gcon"]
    return np.einsum("lk...,kmn...->lmn...", gcon, low)


class Grid:
    """Zone positions and the 2D geometry tables of one problem.

    Tables live on the padded 2D index grid [n2+6, n1+6]. A face table at
    padded index (j, i) describes the *lower* face of zone (j, i) in its
    direction: F1 at x1 = x1min + (i-3) dx1, F2 at x2 = x2min + (j-3) dx2. The
    x3 faces share the zone-centre geometry (nothing depends on x3).
    """

    def __init__(self, prm):
        self.prm = prm
        self.n = (prm["n1"], prm["n2"], prm["n3"])
        self.dx = tuple((prm[f"x{d}max"] - prm[f"x{d}min"]) / prm[f"n{d}"] for d in (1, 2, 3))
        self.kerr = prm["coords"] != MINKOWSKI_CART
        i = np.arange(-NG, prm["n1"] + NG)
        j = np.arange(-NG, prm["n2"] + NG)
        x1c = prm["x1min"] + (i + 0.5) * self.dx[0]
        x2c = prm["x2min"] + (j + 0.5) * self.dx[1]
        x1f = prm["x1min"] + i * self.dx[0]
        x2f = prm["x2min"] + j * self.dx[1]
        X1c, X2c = np.meshgrid(x1c, x2c)
        X1f, X2f = np.meshgrid(x1f, x2f)
        self.x1c, self.x2c = X1c, X2c
        self.cent = metric(X1c, X2c, prm)
        self.face = {1: metric(X1f, X2c, prm), 2: metric(X1c, X2f, prm), 3: self.cent}
        self.conn = connection(X1c, X2c, prm)
        self.r = np.exp(X1c) if self.kerr else None
