"""Primitive reconstruction at zone faces (oracle).

MC (monotonised-central, van Leer): per zone the slope is 0 at an extremum
(Delta- Delta+ <= 0) and otherwise sign(Delta_c) min(2|Delta-|, 2|Delta+|, |Delta_c|),
with Delta- = P_i - P_{i-1}, Delta+ = P_{i+1} - P_i, Delta_c = (P_{i+1} - P_{i-1})/2.
The face states at the lower face of zone i are P_L = P_{i-1} + s_{i-1}/2 and
P_R = P_i - s_i/2.

WENO5 (reading: the point-value form used in HARM-family codes; the paper
names no variant): the value at the right edge of zone i from
(x1..x5) = (P_{i-2} .. P_{i+2}) is sum_k w_k q_k with

  q0 = 3/8 x1 - 5/4 x2 + 15/8 x3,  q1 = -1/8 x2 + 3/4 x3 + 3/8 x4,
  q2 = 3/8 x3 + 3/4 x4 - 1/8 x5,
  beta0 = 13/12 (x1 - 2x2 + x3)^2 + 1/4 (x1 - 4x2 + 3x3)^2
  beta1 = 13/12 (x2 - 2x3 + x4)^2 + 1/4 (x2 - x4)^2
  beta2 = 13/12 (x3 - 2x4 + x5)^2 + 1/4 (3x3 - 4x4 + x5)^2
  alpha_k = d_k / (eps + beta_k)^2,  d = (1/16, 5/8, 5/16),  eps = 1e-26,
  w_k = alpha_k / sum alpha.

The left edge is the same formula on the reversed stencil.
"""

import numpy as np

RECON_MC, RECON_WENO5 = 0, 1
WENO_EPS = 1e-26


def mc_slope(pm, p0, pp):
    dm = p0 - pm
    dp = pp - p0
    dc = 0.5 * (pp - pm)
    mag = np.minimum(np.minimum(2.0 * np.abs(dm), 2.0 * np.abs(dp)), np.abs(dc))
    return np.where(dm * dp > 0.0, np.sign(dc) * mag, 0.0)


def weno5_edge(x1, x2, x3, x4, x5):
    q0 = 0.375 * x1 - 1.25 * x2 + 1.875 * x3
    q1 = -0.125 * x2 + 0.75 * x3 + 0.375 * x4
    q2 = 0.375 * x3 + 0.75 * x4 - 0.125 * x5
    b0 = 13.0 / 12.0 * (x1 - 2.0 * x2 + x3) ** 2 + 0.25 * (x1 - 4.0 * x2 + 3.0 * x3) ** 2
    b1 = 13.0 / 12.0 * (x2 - 2.0 * x3 + x4) ** 2 + 0.25 * (x2 - x4) ** 2
    b2 = 13.0 / 12.0 * (x3 - 2.0 * x4 + x5) ** 2 + 0.25 * (3.0 * x3 - 4.0 * x4 + x5) ** 2
    a0 = (1.0 / 16.0) / (WENO_EPS + b0) ** 2
    a1 = (5.0 / 8.0) / (WENO_EPS + b1) ** 2
    a2 = (5.0 / 16.0) / (WENO_EPS + b2) ** 2
    return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2)


def _take(P, axis, start, stop):
    sl = [slice(None)] * P.ndim
    sl[axis] = slice(start, stop)
    return P[tuple(sl)]


def reconstruct(P, axis, recon, f0, f1):
    """Face states (P_L, P_R) at the lower faces of zones f0..f1-1 along ``axis``.

    ``P`` must hold at least 2 (MC) or 3 (WENO5) zones below f0 and 1 (MC) or 2
    (WENO5) zones at or above f1.
    """
    t = lambda o: _take(P, axis, f0 + o, f1 + o)
    if recon == RECON_MC:
        # zone f-1 (left of the face) and zone f (right of the face)
        left = t(-1) + 0.5 * mc_slope(t(-2), t(-1), t(0))
        right = t(0) - 0.5 * mc_slope(t(-1), t(0), t(1))
    elif recon == RECON_WENO5:
        left = weno5_edge(t(-3), t(-2), t(-1), t(0), t(1))
        right = weno5_edge(t(2), t(1), t(0), t(-1), t(-2))
    else:
        raise ValueError(f"unknown reconstruction {recon}")
    return left, right
