"""Un-magnetised spherical (Michel) accretion on an MKS grid.

The Bondi problem of the Tests section. The relativistic polytropic solution
with sonic point r_c: with n = 1/(gamma-1),

  u_c^2 = 1/(2 r_c),  V_c^2 = u_c^2/(1 - 3 u_c^2),  T_c = n V_c^2 / ((n+1)(1 - n V_c^2)),
  C1 = u_c r_c^2 T_c^n,  C2 = (1 + (n+1) T_c)^2 (1 - 2/r_c + u_c^2),

and at each r the temperature T solves (1 + (n+1)T)^2 (1 - 2/r + C1^2/(r^4 T^(2n))) = C2,
taking the subsonic (large-T) root outside r_c and the supersonic root inside.
Then rho = (T/T_c)^n, u = n rho T, u^r = -C1/(r^2 T^n), and u^t follows from the
Kerr-Schild normalisation with u^theta = u^phi = 0. For a = 0 this is a
stationary solution; for a != 0 it is only used as a workload.

The outer x1 ghosts carry the analytic solution (Dirichlet boundary).
"""

import math

import numpy as np

from .params import (NG, KERR_MKS, RECON_MC, FP64, BC_OUTFLOW, BC_DIRICHLET, BC_POLAR,
                     BC_PERIODIC, base_problem, kerr_grid_extent)
from .kerr import theta_map, centres, ks_gcov, ks_to_code_velocity, normal_frame_velocity_ks


def michel_constants(rc, gam):
    n = 1.0 / (gam - 1.0)
    uc2 = 1.0 / (2.0 * rc)
    vc2 = uc2 / (1.0 - 3.0 * uc2)
    tc = n * vc2 / ((n + 1.0) * (1.0 - n * vc2))
    c1 = math.sqrt(uc2) * rc * rc * tc ** n
    c2 = (1.0 + (n + 1.0) * tc) ** 2 * (1.0 - 2.0 / rc + uc2)
    return n, tc, c1, c2


def michel_temperature(r, rc, gam):
    """Temperature T(r) of the Michel solution by bisection on the right branch."""
    n, tc, c1, c2 = michel_constants(rc, gam)
    r = np.asarray(r, dtype=np.float64)

    def resid(t, r):
        return (1.0 + (n + 1.0) * t) ** 2 * (1.0 - 2.0 / r + c1 * c1 / (r ** 4 * t ** (2.0 * n))) - c2

    # the residual has a single minimum in T: locate it by golden-section search
    # in log T, then bisect the wanted branch between the minimum and a far end
    out = np.empty_like(r)
    gr = 0.5 * (math.sqrt(5.0) - 1.0)
    for idx, rr in np.ndenumerate(r):
        a_, b_ = -30.0, 5.0
        for _ in range(200):
            c_ = b_ - gr * (b_ - a_)
            d_ = a_ + gr * (b_ - a_)
            if resid(math.exp(c_), rr) < resid(math.exp(d_), rr):
                b_ = d_
            else:
                a_ = c_
        tmin = math.exp(0.5 * (a_ + b_))
        if resid(tmin, rr) >= 0.0:
            out[idx] = tmin          # the two roots merge at the sonic point
            continue
        lo, hi = (tmin, 1e5) if rr > rc else (1e-30, tmin)
        flo = resid(lo, rr)
        for _ in range(300):
            mid = math.sqrt(lo * hi)
            fm = resid(mid, rr)
            if (fm > 0) == (flo > 0):
                lo, flo = mid, fm
            else:
                hi = mid
        out[idx] = math.sqrt(lo * hi)
    return out


def bondi(n1=128, n2=128, n3=1, a=0.0, rc=8.0, gam=4.0 / 3.0, r_out=40.0,
          recon=RECON_MC, precision=FP64):
    x1min, x1max = kerr_grid_extent(n1, a, r_out)
    prm = base_problem(
        n1, n2, n3, coords=KERR_MKS, a=a, gam=gam, hslope=1.0,
        x1min=x1min, x1max=x1max, x2min=0.0, x2max=1.0, x3min=0.0, x3max=2.0 * math.pi,
        bc=[[BC_OUTFLOW, BC_DIRICHLET], [BC_POLAR, BC_POLAR], [BC_PERIODIC, BC_PERIODIC]],
        floors=1, recon=recon, precision=precision, _name="bondi", _rc=rc)
    x1c, _ = centres(prm, 1)
    x2c, _ = centres(prm, 2)
    X1, X2 = np.meshgrid(x1c, x2c)
    th, dth1, dth2 = theta_map(X1, X2, prm)
    r1 = np.exp(x1c)
    n, tc, c1, _ = michel_constants(rc, gam)
    T1 = michel_temperature(r1, rc, gam)
    T = np.broadcast_to(T1, X1.shape)
    r = np.exp(X1)
    rho = (T / tc) ** n
    uu = n * rho * T
    ur = -c1 / (r * r * T ** n)
    g = ks_gcov(r, th, a)
    # g_tt (u^t)^2 + 2 g_tr u^t u^r + g_rr (u^r)^2 + 1 = 0, future root (stable form)
    qa = g[0, 0]
    qb = 2.0 * g[0, 1] * ur
    qc = g[1, 1] * ur * ur + 1.0
    ut = 2.0 * qc / (-qb + np.sqrt(qb * qb - 4.0 * qa * qc))
    vr, vth, vph = normal_frame_velocity_ks(ut, ur, 0.0 * ur, 0.0 * ur, r, th, a)
    v1, v2, v3 = ks_to_code_velocity(vr, vth, vph, r, dth1, dth2)

    P = np.zeros((8, n3 + 2 * NG, n2 + 2 * NG, n1 + 2 * NG))
    for v, q in enumerate((rho, uu, v1, v2, v3)):
        P[v] = q[None, :, :]
    # zero every ghost except the outer-x1 (Dirichlet) ones
    keep = np.zeros(P.shape[1:], dtype=bool)
    keep[NG:NG + n3, NG:NG + n2, NG:NG + n1] = True
    keep[NG:NG + n3, NG:NG + n2, NG + n1:] = True
    P[:, ~keep] = 0.0
    return prm, P
