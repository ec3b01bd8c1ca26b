"""Magnetic fields with a known discrete divergence.

Inputs for checking the corner-centred divergence monitor against closed
forms. Each generator lays down sqrt(-g) B^d as a product of sines and cosines
of the code coordinates, so that the corner differences and the transverse
averages of the monitor reduce to exact trigonometric identities:

  [sin 2 pi m x_(i) - sin 2 pi m x_(i-1)] / dx = 2 cos(2 pi m x_c) sin(pi m dx) / dx,
  [cos 2 pi m y_(j) + cos 2 pi m y_(j-1)] / 2 = cos(2 pi m y_c) cos(pi m dy),

with x_(i) the zone centres and x_c the corner between them. The closed form
of the divergence at every corner is returned beside the state. The fluid part
is a uniform state at rest; it plays no role in the divergence.
"""

import math

import numpy as np

from .params import NG, KERR_FMKS, BC_OUTFLOW, BC_POLAR, BC_PERIODIC, base_problem, kerr_grid_extent
from .kerr import theta_map, centres


def _corner_coords(prm, d, periodic):
    """Code coordinates of the corners the monitor reports along direction d
    (lower corner of each zone, the first one dropped on a non-periodic edge)."""
    n = prm[f"n{d}"]
    lo, hi = prm[f"x{d}min"], prm[f"x{d}max"]
    dx = (hi - lo) / n
    idx = np.arange(0 if periodic else 1, n)
    return lo + idx * dx, dx


def sine_box(n1=16, n2=8, n3=4, terms=((1, 1, 1.0, 0),)):
    """Minkowski periodic box on [0, 1)^3 with

      B^d = sum over the terms (d, m, c, t) with that d of
            c sin(2 pi m x_d) cos(2 pi x_t)      (t = 0: no cosine factor),

    d, t in {1, 2, 3}, t != d. Returns (prm, P, div) with div[k, j, i] the exact
    corner divergence at corner (i - 1/2, j - 1/2, k - 1/2).
    """
    prm = base_problem(n1, n2, n3, _name="sine_box")
    n = {1: n1, 2: n2, 3: n3}
    xc = {d: (np.arange(n[d]) + 0.5) / n[d] for d in (1, 2, 3)}
    xk = {d: np.arange(n[d]) / n[d] for d in (1, 2, 3)}
    shape = (n3, n2, n1)
    axis = {1: 2, 2: 1, 3: 0}

    def along(vals, d):
        s = [1, 1, 1]
        s[axis[d]] = -1
        return np.asarray(vals).reshape(s)

    P = np.zeros((8, n3 + 2 * NG, n2 + 2 * NG, n1 + 2 * NG))
    P[0] = 1.0
    P[1] = 1.0
    div = np.zeros(shape)
    for (d, m, c, t) in terms:
        dx = 1.0 / n[d]
        b = c * along(np.sin(2 * math.pi * m * xc[d]), d)
        dv = c * along(2.0 * np.cos(2 * math.pi * m * xk[d]) * math.sin(math.pi * m * dx) / dx, d)
        if t:
            b = b * along(np.cos(2 * math.pi * xc[t]), t)
            dv = dv * along(np.cos(2 * math.pi * xk[t]) * math.cos(math.pi / n[t]), t)
        P[4 + d, NG:NG + n3, NG:NG + n2, NG:NG + n1] += np.broadcast_to(b, shape)
        div = div + np.broadcast_to(dv, shape)
    return prm, P, div


def sine_kerr(n1=32, n2=16, n3=4, a=0.9375, r_out=40.0, m=1, c=1.0):
    """Kerr FMKS grid (outflow x1, polar x2, periodic x3) carrying

      sqrt(-g) B^1 = c sin(2 pi m (x1 - x1min) / L1),  B^2 = B^3 = 0,

    with sqrt(-g) = Sigma |sin theta| r dtheta/dx2 the code-coordinate volume
    element of Kerr-Schild (r = exp x1). Returns (prm, P, div) with div the exact
    corner divergence at the corners the monitor reports (x1 and x2 edges
    excluded): [n3, n2 - 1, n1 - 1].
    """
    x1min, x1max = kerr_grid_extent(n1, a, r_out)
    prm = base_problem(n1, n2, n3, coords=KERR_FMKS, a=a, x1min=x1min, x1max=x1max,
                       x3max=2.0 * math.pi,
                       bc=[[BC_OUTFLOW, BC_OUTFLOW], [BC_POLAR, BC_POLAR], [BC_PERIODIC, BC_PERIODIC]],
                       _name="sine_kerr")
    x1, dx1 = centres(prm, 1, extra=0)
    x2, _ = centres(prm, 2, extra=0)
    X2, X1 = np.meshgrid(x2, x1, indexing="ij")
    th, _, dth2 = theta_map(X1, X2, prm)
    r = np.exp(X1)
    gdet = (r * r + a * a * np.cos(th) ** 2) * np.abs(np.sin(th)) * r * dth2
    L1 = x1max - x1min
    P = np.zeros((8, n3 + 2 * NG, n2 + 2 * NG, n1 + 2 * NG))
    P[0] = 1.0
    P[1] = 1.0
    G1 = c * np.sin(2 * math.pi * m * (X1 - x1min) / L1)
    P[5, NG:NG + n3, NG:NG + n2, NG:NG + n1] = (G1 / gdet)[None]
    xk, _ = _corner_coords(prm, 1, periodic=False)
    d1 = c * 2.0 * np.cos(2 * math.pi * m * (xk - x1min) / L1) * math.sin(math.pi * m * dx1 / L1) / dx1
    div = np.broadcast_to(d1[None, None, :], (n3, n2 - 1, n1 - 1))
    return prm, P, np.array(div)
