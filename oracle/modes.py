"""Linear MHD eigenmodes of a uniform state at rest (oracle).

For a plane wave dP exp(i (k.x - omega t)) on a uniform background, the
linearised conservation law M dP_t + sum_d A_d dP_d = 0 with M = dU/dP and
A_d = dF^d/dP gives the generalised eigenproblem

  (sum_d k_d A_d) R = omega M R.

The Jacobians are taken by complex-step differentiation of the oracle's own
conserved variables and fluxes in flat space. The Tests section evolves such
modes as the 3D convergence problem.
"""

import numpy as np

from .physics import fluid_state, flux, conserved

H = 1e-20


def _flat_geo():
    eta = np.diag([-1.0, 1.0, 1.0, 1.0]).astype(complex)
    return dict(gcov=eta, gcon=eta, gdet=1.0, alpha=1.0)


def jacobians(P0, gam):
    geo = _flat_geo()
    M = np.zeros((8, 8))
    A = np.zeros((3, 8, 8))
    for j in range(8):
        P = np.asarray(P0, dtype=complex).copy()
        P[j] += 1j * H
        st = fluid_state(P, geo, gam)
        M[:, j] = np.imag(conserved(st, 1.0)) / H
        for d in range(1, 4):
            A[d - 1, :, j] = np.imag(flux(st, d, 1.0)) / H
    return M, A


def eigenmodes(P0, gam, kvec):
    """(omega, R) for the slow, Alfven and fast modes with omega > 0.

    R is normalised to unit 2-norm with its largest-magnitude component real
    and positive.
    """
    M, A = jacobians(P0, gam)
    k = 2.0 * np.pi * np.asarray(kvec, dtype=float)
    K = np.einsum("d,dij->ij", k, A)
    w, V = np.linalg.eig(np.linalg.solve(M, K))
    order = [i for i in np.argsort(w.real) if w[i].real > 1e-8]
    out = {}
    for name, i in zip(("slow", "alfven", "fast"), order):
        R = V[:, i]
        R = R / np.linalg.norm(R)
        m = np.argmax(np.abs(R))
        R = R * (abs(R[m]) / R[m])
        out[name] = (float(w[i].real), R)
    return out
