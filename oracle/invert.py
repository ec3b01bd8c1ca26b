"""Conserved -> primitive inversion by the 1D_W scheme (oracle).

Implementation Notes section: conserved variables are stepped and inverted to
primitives numerically with the 1D_W scheme of Noble et al. (2006). Per zone,
with U~ = U / sqrt(-g) and the normal observer n_mu = (-alpha, 0, 0, 0):

  D = alpha U~_rho,  Q_i = alpha U~_i,  B^i (normal frame) = alpha U~_B^i
  Q.n + D = U~_E + (alpha - 1) U~_rho - alpha g^{ti} Q_i
  Q~^i = gamma^{ij} Q_j,  Q~^2 = Q_i Q~^i,  gamma^{ij} = g^{ij} + alpha^2 g^{ti} g^{tj}
  Q.B = Q_i B^i,  B^2 = g_ij B^i B^j

W = rho h Gamma^2 is the root of

  f(W) = Q.n + W - p + B^2 (1 + v^2)/2 - (Q.B)^2/(2 W^2) = 0,
  v^2(W) = [Q~^2 W^2 + (Q.B)^2 (B^2 + 2W)] / [(B^2 + W)^2 W^2],
  p = (gamma-1)/gamma [W (1 - v^2) - D sqrt(1 - v^2)],

after which Gamma = 1/sqrt(1 - v^2), rho = D/Gamma, u = (W/Gamma^2 - rho)/gamma,
u~^i = Gamma/(W + B^2) [Q~^i + (Q.B) B^i / W] and B^i = U~_B^i.

Readings (the paper names the scheme only):
* the unknown is W' = W - D, and W(1 - v^2) - D sqrt(1 - v^2) is evaluated as
  W'(1 - v^2) - D s v^2/(1 + s) with s = sqrt(1 - v^2), so nothing cancels at
  small u/rho or small v; likewise Q~ uses the spatial metric gamma^{ij} directly;
* Newton with the analytic derivative, from the guess primitives; a step that
  would make W <= 0 halves W instead; v^2 is clamped to [0, 1 - 1e-12] inside
  the iteration, and where the clamp is active its (zero) derivative is used,
  so a guess with v^2(W) >= 1 steps straight out of that region; converged
  once |dW'| <= 1e-8 W, after which two more Newton steps are taken; at most
  50 iterations;
* failure = never converged, W <= 0, final v^2 >= 1 - 1e-12, or a non-finite
  value. A failed zone keeps the guess's hydro primitives (for the fixup).
"""

import numpy as np

TOL = 1e-8
EXTRA = 2
MAXIT = 50
V2MAX = 1.0 - 1e-12


def _prepare(U, geo):
    gcov, gcon, gdet, alpha = geo["gcov"], geo["gcon"], geo["gdet"], geo["alpha"]
    Ut = U / gdet
    D = alpha * Ut[0]
    Q = [alpha * Ut[2], alpha * Ut[3], alpha * Ut[4]]
    Bn = [alpha * Ut[5], alpha * Ut[6], alpha * Ut[7]]
    qn_d = Ut[1] + (alpha - 1.0) * Ut[0] - alpha * sum(gcon[0, i + 1] * Q[i] for i in range(3))
    a2 = alpha * alpha
    gsp = [[gcon[i + 1, j + 1] + a2 * gcon[0, i + 1] * gcon[0, j + 1] for j in range(3)]
           for i in range(3)]
    qtil = [sum(gsp[i][j] * Q[j] for j in range(3)) for i in range(3)]
    qtsq = sum(Q[i] * qtil[i] for i in range(3))
    qdb = sum(Q[i] * Bn[i] for i in range(3))
    bsq = sum(gcov[i + 1, j + 1] * Bn[i] * Bn[j] for i in range(3) for j in range(3))
    return Ut, D, Bn, qn_d, qtil, qtsq, qdb, bsq


def _v2(W, qtsq, qdb, bsq):
    return (qtsq * W * W + qdb * qdb * (bsq + 2.0 * W)) / ((bsq + W) ** 2 * W * W)


def _f_df(x, D, qn_d, qtsq, qdb, bsq, gam):
    W = x + D
    v2raw = _v2(W, qtsq, qdb, bsq)
    v2 = np.clip(v2raw, 0.0, V2MAX)
    s = np.sqrt(1.0 - v2)
    wmr = x * (1.0 - v2) - D * s * v2 / (1.0 + s)
    gf = (gam - 1.0) / gam
    p = gf * wmr
    f = qn_d + x - p + 0.5 * bsq * (1.0 + v2) - 0.5 * qdb * qdb / (W * W)
    dv2 = (-2.0 * (qtsq * W ** 3 + qdb * qdb * (3.0 * W * W + 3.0 * W * bsq + bsq * bsq))
           / ((bsq + W) ** 3 * W ** 3))
    dv2 = np.where((v2raw > V2MAX) | (v2raw < 0.0), 0.0, dv2)    # derivative of the clamp
    dp = gf * ((1.0 - v2) + (-W + D / (2.0 * s)) * dv2)
    df = 1.0 - dp + 0.5 * bsq * dv2 + qdb * qdb / W ** 3
    return f, df


def invert(U, guess, geo, gam, maxit=MAXIT):
    """Return (P, failed) for conserved U [8, ...] and guess primitives [8, ...]."""
    Ut, D, Bn, qn_d, qtil, qtsq, qdb, bsq = _prepare(U, geo)
    gcov = geo["gcov"]
    v = guess[2:5]
    lor2 = 1.0 + sum(gcov[i + 1, j + 1] * v[i] * v[j] for i in range(3) for j in range(3))
    x = (guess[0] + gam * guess[1]) * lor2 - D
    x = np.broadcast_to(x, np.broadcast(x, D, qtsq).shape).copy()
    extra = np.full(x.shape, -1, dtype=np.int64)     # -1: not yet converged
    with np.errstate(all="ignore"):
        for _ in range(maxit):
            active = extra < EXTRA
            if not active.any():
                break
            f, df = _f_df(x, D, qn_d, qtsq, qdb, bsq, gam)
            dx = -f / df
            xn = x + dx
            xn = np.where(xn + D <= 0.0, 0.5 * (x + D) - D, xn)
            x = np.where(active, xn, x)
            hit = active & (extra < 0) & (np.abs(dx) <= TOL * np.abs(x + D))
            extra = np.where(active & (extra >= 0), extra + 1, extra)
            extra = np.where(hit, 0, extra)
        W = x + D
        v2 = _v2(W, qtsq, qdb, bsq)
        failed = (extra < 0) | (W <= 0.0) | (v2 >= V2MAX) | ~np.isfinite(v2) | ~np.isfinite(W)
        v2c = np.clip(v2, 0.0, V2MAX)
        s = np.sqrt(1.0 - v2c)
        lor = 1.0 / s
        rho = D * s
        u = (x * (1.0 - v2c) - D * s * v2c / (1.0 + s)) / gam
        fac = lor / (W + bsq)
        vel = [fac * (qtil[i] + qdb * Bn[i] / W) for i in range(3)]
    P = np.array(np.broadcast_arrays(rho, u, vel[0], vel[1], vel[2], Ut[5], Ut[6], Ut[7]))
    bad = failed | ~np.all(np.isfinite(P[:5]), axis=0)
    g = np.broadcast_to(guess, P.shape)
    P[:5] = np.where(bad, g[:5], P[:5])
    return P, bad
