"""Point physics of ideal GRMHD in HARM variables (oracle).

Units GM = c = 1 with the factor sqrt(4 pi) absorbed into B, so the magnetic
pressure is b^2/2 (Implementation Notes section). Ideal gas p = (gamma-1) u.

From primitives (rho, u, u~^i, B^i), with u~ the velocity relative to the
normal observer n_mu = (-alpha, 0, 0, 0):

  Gamma = sqrt(1 + g_ij u~^i u~^j),  u^t = Gamma/alpha,  u^i = u~^i - Gamma alpha g^{ti}
  b^t = B^i u_i,  b^i = (B^i + b^t u^i)/u^t
  T^mu_nu = (w + b^2) u^mu u_nu + (p + b^2/2) delta^mu_nu - b^mu b_nu,  w = rho + u + p

and the conserved variables / fluxes in direction d (d = 0 gives U):

  F^d = sqrt(-g) (rho u^d, T^d_t + rho u^d, T^d_i, b^i u^d - b^d u^i)

The rest-mass flux is added to the energy component (HARM convention), and
the B part of U is sqrt(-g) B^i exactly.

Every function takes component-first arrays ([8, ...] primitives, [4, 4, ...]
metric) and is written so complex inputs work (used for complex-step
Jacobians of the linear-mode eigenproblem).
"""

import numpy as np


def fluid_state(P, geo, gam):
    """Four-vectors and scalars of the fluid at each point."""
    gcov, gcon, alpha = geo["gcov"], geo["gcon"], geo["alpha"]
    rho, u = P[0], P[1]
    v = P[2:5]
    B = P[5:8]
    qsq = sum(gcov[i + 1, j + 1] * v[i] * v[j] for i in range(3) for j in range(3))
    lor = np.sqrt(1.0 + qsq)
    ucon = [lor / alpha] + [v[i] - lor * alpha * gcon[0, i + 1] for i in range(3)]
    ucov = [sum(gcov[m, n] * ucon[n] for n in range(4)) for m in range(4)]
    bt = sum(B[i] * ucov[i + 1] for i in range(3))
    bcon = [bt] + [(B[i] + bt * ucon[i + 1]) / ucon[0] for i in range(3)]
    bcov = [sum(gcov[m, n] * bcon[n] for n in range(4)) for m in range(4)]
    bsq = sum(bcon[m] * bcov[m] for m in range(4))
    p = (gam - 1.0) * u
    return dict(rho=rho, u=u, p=p, w=rho + u + p, B=B, lorentz=lor,
                ucon=ucon, ucov=ucov, bcon=bcon, bcov=bcov, bsq=bsq)


def stress(st, mu, nu):
    """T^mu_nu."""
    d = 1.0 if mu == nu else 0.0
    return ((st["w"] + st["bsq"]) * st["ucon"][mu] * st["ucov"][nu]
            + (st["p"] + 0.5 * st["bsq"]) * d - st["bcon"][mu] * st["bcov"][nu])


def flux(st, d, gdet):
    """sqrt(-g) F^d for d in 1..3, [8, ...]."""
    ud = st["ucon"][d]
    mass = st["rho"] * ud
    out = [mass, stress(st, d, 0) + mass, stress(st, d, 1), stress(st, d, 2), stress(st, d, 3)]
    for i in range(1, 4):
        out.append(st["bcon"][i] * ud - st["bcon"][d] * st["ucon"][i])
    return np.array([gdet * q for q in np.broadcast_arrays(*out)])


def conserved(st, gdet):
    """U = sqrt(-g) F^t, with the B part sqrt(-g) B^i, [8, ...]."""
    ut = st["ucon"][0]
    mass = st["rho"] * ut
    out = [mass, stress(st, 0, 0) + mass, stress(st, 0, 1), stress(st, 0, 2), stress(st, 0, 3),
           st["B"][0], st["B"][1], st["B"][2]]
    return np.array([gdet * q for q in np.broadcast_arrays(*out)])


def signal_speeds(st, geo, d, gam):
    """Largest and smallest fast-magnetosonic speeds dx^d/dt.

    With v_A^2 = b^2/(b^2 + w), c_s^2 = gamma p / w and c^2 = v_A^2 + c_s^2 (1 - v_A^2)
    (the fast speed across the field, an upper bound for every direction), the
    speeds are the roots of A l^2 + B l + C = 0 with
      A = (u^t)^2 - c^2 (g^tt + (u^t)^2)
      B = -2 [u^t u^d - c^2 (g^td + u^t u^d)]
      C = (u^d)^2 - c^2 (g^dd + (u^d)^2).
    """
    gcon = geo["gcon"]
    cs2 = gam * st["p"] / st["w"]
    va2 = st["bsq"] / (st["bsq"] + st["w"])
    c2 = va2 + cs2 * (1.0 - va2)
    ut, ud = st["ucon"][0], st["ucon"][d]
    A = ut * ut - c2 * (gcon[0, 0] + ut * ut)
    B = -2.0 * (ut * ud - c2 * (gcon[0, d] + ut * ud))
    C = ud * ud - c2 * (gcon[d, d] + ud * ud)
    disc = np.sqrt(np.maximum(B * B - 4.0 * A * C, 0.0))
    vp = (-B + disc) / (2.0 * A)
    vm = (-B - disc) / (2.0 * A)
    return np.maximum(vp, vm), np.minimum(vp, vm)
