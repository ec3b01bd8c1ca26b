"""Magnetised spherical accretion on a Cartesian Kerr-Schild box.

This workload uses a spacetime whose metric depends on all three code
coordinates. The code coordinates are the Cartesian Kerr-Schild (x, y, z). The
Implementation Notes treat a new set of coordinates or a new stationary
background as a small change, since only the metric evaluation differs.

* Position. The Boyer-Lindquist-like radius r is the positive root of
  r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0, with cos theta = z / r and
  x + i y = (r + i a) sin theta e^{i phi}. This map takes the spherical
  Kerr-Schild metric of ``kerr.ks_gcov`` to the Cartesian form
  eta + f l l.
* Flow. It is the Michel solution of ``bondi`` (u^r(r), theta and phi
  components zero). The sonic point is r_c and the density is 1 there.
* Field. It is radial, B^r = b0 / (r^2 + a^2 cos^2 theta), so sqrt(-g) B^r is
  independent of r (divergence free). With a = 0 both flow and field are
  stationary: a radial field exerts no force on a radial flow.
* Conversion to Cartesian. Contravariant components go through
  d(x, y, z)/dr = (sin theta cos phi, sin theta sin phi, cos theta). The
  normal-frame velocity is u~^i = u^i - u^t g^{ti} / g^{tt}, with g^{mu nu}
  the numerical inverse of this module's own Cartesian metric.
* Boundaries. They are Dirichlet on all six sides, so the ghost zones hold
  the solution.

T(r) comes from a vectorised form of the branch search in ``bondi``: a
golden-section search for the minimum of the residual, then bisection on the
wanted side. Grids of more than 2^20 padded zones (benchmark sizes) take T
from 65536 log-spaced radii, interpolated linearly in (log r, log T): relative
error below 2e-11. At a = 0 ``test_oracle_cks`` checks the data against the
Schwarzschild form of the solution.
"""

import math

import numpy as np

from .params import (NG, KERR_CKS, RECON_MC, FP64, BC_DIRICHLET, base_problem)
from .kerr import ks_gcov, centres
from .bondi import michel_constants


def cks_point(x, y, z, a):
    """(r, theta, phi) of a Cartesian Kerr-Schild point."""
    h = 0.5 * (x * x + y * y + z * z - a * a)
    r = np.sqrt(h + np.sqrt(h * h + a * a * z * z))
    th = np.arccos(np.clip(z / r, -1.0, 1.0))
    w = (x + 1j * y) / (r + 1j * a)
    return r, th, np.angle(w)


def cks_metric(x, y, z, a):
    """eta + f l l in (t, x, y, z), [4, 4, ...]."""
    r, _, _ = cks_point(x, y, z, a)
    f = 2.0 * r ** 3 / (r ** 4 + a * a * z * z)
    den = r * r + a * a
    l = [np.ones_like(r), (r * x + a * y) / den, (r * y - a * x) / den, z / r]
    g = np.array([[f * l[m] * l[n] for n in range(4)] for m in range(4)])
    for m in range(4):
        g[m, m] += -1.0 if m == 0 else 1.0
    return g


def michel_temperature_vec(r, rc, gam):
    """T(r) of the Michel solution for an array of radii (the search of
    ``bondi.michel_temperature``, elementwise on arrays)."""
    n, tc, c1, c2 = michel_constants(rc, gam)
    r = np.asarray(r, dtype=np.float64)

    def resid(t):
        return (1.0 + (n + 1.0) * t) ** 2 * (1.0 - 2.0 / r + c1 * c1 / (r ** 4 * t ** (2.0 * n))) - c2

    gr = 0.5 * (math.sqrt(5.0) - 1.0)
    lo = np.full(r.shape, -30.0)
    hi = np.full(r.shape, 5.0)
    for _ in range(200):
        c = hi - gr * (hi - lo)
        d = lo + gr * (hi - lo)
        left = resid(np.exp(c)) < resid(np.exp(d))
        hi = np.where(left, d, hi)
        lo = np.where(left, lo, c)
    tmin = np.exp(0.5 * (lo + hi))
    merged = resid(tmin) >= 0.0
    outside = r > rc
    blo = np.where(outside, tmin, 1e-30)
    bhi = np.where(outside, 1e5, tmin)
    flo = resid(blo)
    for _ in range(300):
        mid = np.sqrt(blo * bhi)
        fm = resid(mid)
        same = (fm > 0) == (flo > 0)
        blo = np.where(same, mid, blo)
        flo = np.where(same, fm, flo)
        bhi = np.where(same, bhi, mid)
    return np.where(merged, tmin, np.sqrt(blo * bhi))


def cks_bondi(n1=24, n2=20, n3=16, a=0.9375, rc=8.0, gam=4.0 / 3.0, b0=15.0,
              box=((6.0, 14.0), (-4.0, 4.0), (-3.0, 5.0)), recon=RECON_MC, precision=FP64, floors=1):
    (x1lo, x1hi), (x2lo, x2hi), (x3lo, x3hi) = box
    prm = base_problem(
        n1, n2, n3, coords=KERR_CKS, a=a, gam=gam,
        x1min=x1lo, x1max=x1hi, x2min=x2lo, x2max=x2hi, x3min=x3lo, x3max=x3hi,
        bc=[[BC_DIRICHLET, BC_DIRICHLET]] * 3, floors=floors, recon=recon, precision=precision,
        _name="cks_bondi", _rc=rc)
    xc = [centres(prm, d)[0] for d in (1, 2, 3)]
    Z, Y, X = np.meshgrid(xc[2], xc[1], xc[0], indexing="ij")
    r, th, ph = cks_point(X, Y, Z, a)
    if np.min(r) <= 1.0 + math.sqrt(1.0 - a * a):
        raise ValueError("the box (with ghosts) must lie outside the horizon")
    n, tc, c1, _ = michel_constants(rc, gam)
    if r.size <= 1 << 20:
        T = michel_temperature_vec(r, rc, gam)
    else:
        rs = np.geomspace(r.min(), r.max(), 1 << 16)
        T = np.exp(np.interp(np.log(r), np.log(rs), np.log(michel_temperature_vec(rs, rc, gam))))
    rho = (T / tc) ** n
    uu = n * rho * T
    ur = -c1 / (r * r * T ** n)
    g = ks_gcov(r, th, a)
    qa = g[0, 0]
    qb = 2.0 * g[0, 1] * ur
    qc = g[1, 1] * ur * ur + 1.0
    ut = 2.0 * qc / (-qb + np.sqrt(qb * qb - 4.0 * qa * qc))
    dr = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    gc = np.moveaxis(np.linalg.inv(np.moveaxis(cks_metric(X, Y, Z, a), (0, 1), (-2, -1))), (-2, -1), (0, 1))
    vt = [dr[i] * ur - ut * gc[0, i + 1] / gc[0, 0] for i in range(3)]
    br = b0 / (r * r + a * a * np.cos(th) ** 2)
    P = np.array([rho, uu, vt[0], vt[1], vt[2], dr[0] * br, dr[1] * br, dr[2] * br])
    return prm, P
