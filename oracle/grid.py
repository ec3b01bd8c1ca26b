"""Coordinates, metric and connection (oracle).

Implementation Notes section: every metric-dependent quantity is evaluated
numerically from the line element in analytic form, and the coordinates act
as static mesh refinement. Here:

* Minkowski: Cartesian code coordinates, g = diag(-1, 1, 1, 1).
* Kerr, Cartesian Kerr-Schild: code coordinates (x1, x2, x3) = (x, y, z) and
  g = eta + f l l (the Kerr-Schild form of the Kerr metric, a change of
  background spacetime coordinates the Implementation Notes call trivial), with
  r the Boyer-Lindquist-like radius of the point, the positive root of
  r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0 (R^2 = x^2 + y^2 + z^2),
  f = 2 r^3 / (r^4 + a^2 z^2) and the null covector
  l = (1, (r x + a y)/(r^2 + a^2), (r y - a x)/(r^2 + a^2), z/r).
  Every metric quantity depends on all three code coordinates, so the tables
  are 3D.
* Kerr: Kerr-Schild (t, r, theta, phi) with code coordinates r = exp(x1),
  theta = theta(x1, x2) (MKS, or "funky" MKS which blends in a polynomial
  theta_J(x2) that flattens the resolution near the poles), phi = x3.
  g_code = J^T g_KS J with the analytic Jacobian J = d(t,r,theta,phi)/d(x0..x3).
* g^{mu nu} is the numerical inverse, sqrt(-g) the square root of minus the
  numerical determinant, alpha = 1/sqrt(-g^{tt}).
* The connection Gamma^l_{mn} = g^{lk} Gamma_{kmn}, Gamma_{kmn} =
  (d_n g_km + d_m g_kn - d_k g_mn)/2, with the derivatives taken by centred
  differences of g_code in x1 and x2 (step 1e-5); d_t = d_x3 = 0 (in
  Cartesian Kerr-Schild also x3 is differenced; d_t = 0).

Reading (the paper gives no formula for the coordinates): the MKS/FMKS maps of
the HARM literature, with h = 0.3, x_t = 0.82, alpha = 14, s = 0.5; |sin theta|
is kept >= 1e-20 inside the metric so that faces on the polar axis keep an
invertible metric.
"""

import numpy as np

NG = 3
MINKOWSKI_CART, KERR_MKS, KERR_FMKS, KERR_CKS = 0, 1, 2, 3
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


def cks_radius(x, y, z, a):
    """r of a Cartesian Kerr-Schild point: r^2 = (R^2 - a^2)/2 + sqrt((R^2 - a^2)^2/4 + a^2 z^2)."""
    h = 0.5 * (x * x + y * y + z * z - a * a)
    return np.sqrt(h + np.sqrt(h * h + a * a * z * z))


def gcov_cks(x, y, z, a):
    """Kerr metric in Cartesian Kerr-Schild coordinates, g = eta + f l l, [4, 4, ...].

    Only +, -, *, / and sqrt, so every value is a fixed sequence of correctly
    rounded operations (the centred differences of the connection multiply a
    one-ulp difference in g by about 1e5)."""
    r = cks_radius(x, y, z, a)
    r2 = r * r
    f = 2.0 * r2 * r / (r2 * r2 + a * a * z * z)
    ra = r2 + a * a
    l = (np.ones_like(r), (r * x + a * y) / ra, (r * y - a * x) / ra, z / r)
    out = np.zeros((4, 4) + np.shape(r))
    for m in range(4):
        for n in range(4):
            out[m, n] = f * l[m] * l[n]
        out[m, m] += -1.0 if m == 0 else 1.0
    return out


def gcov_code(x1, x2, prm, x3=None):
    """Covariant metric in code coordinates at (x1, x2[, x3]), [4, 4, ...]."""
    if prm["coords"] == KERR_CKS:
        return gcov_cks(x1, x2, x3, prm["a"])
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


def metric(x1, x2, prm, x3=None):
    """dict(gcov, gcon, gdet, alpha) at (x1, x2[, x3])."""
    g = gcov_code(x1, x2, prm, x3)
    gm = np.moveaxis(g, (0, 1), (-2, -1))
    gcon = np.moveaxis(np.linalg.inv(gm), (-2, -1), (0, 1))
    gdet = np.sqrt(np.abs(np.linalg.det(gm)))
    alpha = 1.0 / np.sqrt(-gcon[0, 0])
    return dict(gcov=g, gcon=gcon, gdet=gdet, alpha=alpha)


def connection(x1, x2, prm, delta=FD_DELTA, x3=None):
    """Gamma^l_{mn}, [4, 4, 4, ...], from centred differences of g_code."""
    shape = np.shape(x1 + x2 if x3 is None else x1 + x2 + x3)
    dg = np.zeros((4, 4, 4) + shape)      # dg[c, a, b] = d_c g_ab
    if prm["coords"] != MINKOWSKI_CART:
        dg[1] = (gcov_code(x1 + delta, x2, prm, x3) - gcov_code(x1 - delta, x2, prm, x3)) / (2.0 * delta)
        dg[2] = (gcov_code(x1, x2 + delta, prm, x3) - gcov_code(x1, x2 - delta, prm, x3)) / (2.0 * delta)
    if prm["coords"] == KERR_CKS:
        dg[3] = (gcov_code(x1, x2, prm, x3 + delta) - gcov_code(x1, x2, prm, x3 - delta)) / (2.0 * delta)
    # Gamma_{k m n} = (d_n g_km + d_m g_kn - d_k g_mn) / 2
    low = 0.5 * (np.einsum("nkm...->kmn...", dg) + np.einsum("mkn...->kmn...", dg)
                 - np.einsum("kmn...->kmn...", dg))
    gcon = metric(x1, x2, prm, x3)["gcon"]
    return np.einsum("lk...,kmn...->lmn...", gcon, low)


class Grid:
    """Zone positions and the geometry tables of one problem.

    Axisymmetric coordinates (Minkowski, MKS, FMKS): tables live on the padded
    2D index grid [n2+6, n1+6] and broadcast over x3; the x3 faces share the
    zone-centre geometry. Cartesian Kerr-Schild: tables live on the padded 3D
    grid [n3+6, n2+6, n1+6] (``k3`` is True) with a table of its own for the
    x3 faces. A face table at padded index (k, j, i) describes the *lower*
    face of zone (k, j, i) in its direction: F1 at x1 = x1min + (i-3) dx1, F2
    at x2 = x2min + (j-3) dx2, F3 at x3 = x3min + (k-3) dx3.
    """

    def __init__(self, prm):
        self.prm = prm
        self.n = (prm["n1"], prm["n2"], prm["n3"])
        self.dx = tuple((prm[f"x{d}max"] - prm[f"x{d}min"]) / prm[f"n{d}"] for d in (1, 2, 3))
        self.kerr = prm["coords"] != MINKOWSKI_CART
        self.k3 = prm["coords"] == KERR_CKS
        i = np.arange(-NG, prm["n1"] + NG)
        j = np.arange(-NG, prm["n2"] + NG)
        x1c = prm["x1min"] + (i + 0.5) * self.dx[0]
        x2c = prm["x2min"] + (j + 0.5) * self.dx[1]
        x1f = prm["x1min"] + i * self.dx[0]
        x2f = prm["x2min"] + j * self.dx[1]
        if self.k3:
            k = np.arange(-NG, prm["n3"] + NG)
            x3c = prm["x3min"] + (k + 0.5) * self.dx[2]
            x3f = prm["x3min"] + k * self.dx[2]

            def mesh(a1, a2, a3):
                X3, X2, X1 = np.meshgrid(a3, a2, a1, indexing="ij")
                return X1, X2, X3

            C = mesh(x1c, x2c, x3c)
            self.x1c, self.x2c, self.x3c = C
            self.cent = metric(C[0], C[1], prm, C[2])
            F = {1: mesh(x1f, x2c, x3c), 2: mesh(x1c, x2f, x3c), 3: mesh(x1c, x2c, x3f)}
            self.face = {d: metric(X[0], X[1], prm, X[2]) for d, X in F.items()}
            self.conn = connection(C[0], C[1], prm, x3=C[2])
            self.r = cks_radius(C[0], C[1], C[2], prm["a"])
            return
        X1c, X2c = np.meshgrid(x1c, x2c)
        X1f, X2f = np.meshgrid(x1f, x2f)
        self.x1c, self.x2c = X1c, X2c
        self.cent = metric(X1c, X2c, prm)
        self.face = {1: metric(X1f, X2c, prm), 2: metric(X1c, X2f, prm), 3: self.cent}
        self.conn = connection(X1c, X2c, prm)
        self.r = np.exp(X1c) if self.kerr else None

    def sub(self, tab, K, J, I):
        """A table (array or dict of arrays) at padded slices (K, J, I); K is
        ignored by 2D tables, which broadcast over x3."""
        if isinstance(tab, dict):
            return {name: self.sub(v, K, J, I) for name, v in tab.items()}
        return tab[..., K, J, I] if self.k3 else tab[..., J, I]
