"""Pins of the oracle's Cartesian Kerr-Schild geometry and of its step on an
x3-dependent spacetime (Implementation Notes: changing the coordinate system
or the background spacetime is trivial).

* Metric. The oracle's eta + f l l, pulled back through the map
  x + i y = (r + i a) sin theta e^{i phi}, z = r cos theta, equals the
  spherical Kerr-Schild metric of ``problems.kerr``. That is an independent
  transcription and the Jacobian is analytic. Also det g = -1 and l is null.
* Connection. Metric compatibility fixes Gamma uniquely:
  d_c g_ab = Gamma^d_{ca} g_db + Gamma^d_{cb} g_ad. The test checks this with
  metric derivatives from a fourth-order stencil with a step other than the
  oracle's.
* Step. At a = 0 the magnetised Michel flow is stationary, and the oracle's
  deviation from it converges at second order (12^3 -> 24^3 over one time
  span). A wrong sign or index in the x3 part of the geometry leaves an O(1)
  residual instead.
* Tables. They are 3D and differ between x3 planes, and the x3 faces have a
  table of their own.
"""

import numpy as np
import pytest

import oracle
import problems
from oracle import grid as G
from problems.kerr import ks_gcov

A = 0.9375


def jacobian(r, th, ph, a):
    """d(t, x, y, z) / d(t, r, theta, phi) of the Kerr-Schild Cartesian map."""
    s, c = np.sin(th), np.cos(th)
    sp, cp = np.sin(ph), np.cos(ph)
    J = np.zeros((4, 4))
    J[0, 0] = 1.0
    J[1, 1:] = (cp * s, (r * cp - a * sp) * c, (-r * sp - a * cp) * s)
    J[2, 1:] = (sp * s, (r * sp + a * cp) * c, (r * cp - a * sp) * s)
    J[3, 1:] = (c, -r * s, 0.0)
    return J


def test_cks_metric_is_the_kerr_schild_metric_in_cartesian_form():
    rng = np.random.default_rng(5)
    for a in (0.0, 0.5, A):
        for _ in range(20):
            r, th, ph = rng.uniform(2.0, 20.0), rng.uniform(0.1, 3.0), rng.uniform(-np.pi, np.pi)
            x = (r * np.cos(ph) - a * np.sin(ph)) * np.sin(th)
            y = (r * np.sin(ph) + a * np.cos(ph)) * np.sin(th)
            z = r * np.cos(th)
            assert abs(G.cks_radius(x, y, z, a) - r) < 1e-12 * r
            g = G.gcov_cks(np.float64(x), np.float64(y), np.float64(z), a)
            J = jacobian(r, th, ph, a)
            pulled = J.T @ g @ J
            want = ks_gcov(np.float64(r), np.float64(th), a)
            assert np.abs(pulled - want).max() <= 1e-11 * np.abs(want).max()


def test_cks_determinant_and_null_vector():
    prm, _ = problems.cks_bondi(6, 5, 4)
    grid = oracle.Grid(prm)
    assert grid.k3
    assert np.abs(grid.cent["gdet"] - 1.0).max() < 1e-13
    for d in (1, 2, 3):
        assert np.abs(grid.face[d]["gdet"] - 1.0).max() < 1e-13
    # g - eta = f l l has rank one with a null l: (g - eta)^2 = f^2 (l.l) l l = 0 under eta
    g = grid.cent["gcov"]
    eta = np.diag([-1.0, 1.0, 1.0, 1.0])
    h = g - eta[:, :, None, None, None]
    hh = np.einsum("am...,mn,nb...->ab...", h, eta, h)
    assert np.abs(hh).max() < 1e-12 * np.abs(h).max() ** 2


def test_cks_closed_form_inverse_and_lapse():
    """Reading 17's closed forms, which the kernels evaluate instead of a
    numerical inverse: with h = g - eta = f l l and l null, g^-1 = eta - eta h eta
    and the lapse is 1/sqrt(1 + f), f = h_tt (l_t = 1). Checked against the
    oracle's numerical inverse and lapse at the centres and at all faces."""
    prm, _ = problems.cks_bondi(6, 5, 4)
    grid = oracle.Grid(prm)
    eta = np.diag([-1.0, 1.0, 1.0, 1.0])
    for geo in (grid.cent, grid.face[1], grid.face[2], grid.face[3]):
        g = geo["gcov"]
        h = g - eta[:, :, None, None, None]
        closed = eta[:, :, None, None, None] - np.einsum("am,mn...,nb->ab...", eta, h, eta)
        assert np.abs(closed - geo["gcon"]).max() < 1e-13 * np.abs(geo["gcon"]).max()
        assert np.abs(1.0 / np.sqrt(1.0 + h[0, 0]) - geo["alpha"]).max() < 1e-14


def test_cks_connection_is_metric_compatible():
    prm, _ = problems.cks_bondi(6, 5, 4, a=A)
    grid = oracle.Grid(prm)
    pts = [(1, 2, 3), (4, 0, 5), (7, 6, 2), (2, 9, 8)]
    h = 2e-3
    for k, j, i in pts:
        x = np.array([grid.x1c[k, j, i], grid.x2c[k, j, i], grid.x3c[k, j, i]])
        dg = np.zeros((4, 4, 4))
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            f = lambda s: G.gcov_cks(*(x + s * e), A)
            dg[c + 1] = (-f(2) + 8 * f(1) - 8 * f(-1) + f(-2)) / (12 * h)
        gam = grid.conn[:, :, :, k, j, i]
        g = grid.cent["gcov"][:, :, k, j, i]
        rhs = np.einsum("dca,db->cab", gam, g) + np.einsum("dcb,ad->cab", gam, g)
        assert np.abs(rhs - dg).max() < 1e-8, np.abs(rhs - dg).max()


def test_cks_tables_depend_on_x3_and_x3_faces_have_their_own():
    prm, _ = problems.cks_bondi(6, 5, 4)
    grid = oracle.Grid(prm)
    g = grid.cent["gcov"]
    assert g.shape[2:] == (4 + 6, 5 + 6, 6 + 6)
    assert np.abs(g[:, :, 3] - g[:, :, 4]).max() > 1e-3
    assert np.abs(grid.face[3]["gcov"] - g).max() > 1e-3
    assert np.abs(grid.face[1]["gcov"] - g).max() > 1e-3
    # the lower d-face of zone k sits half a zone below its centre: it is the
    # centre of the same zone on a grid shifted down by dx_d / 2
    for d in (1, 2, 3):
        dx = (prm[f"x{d}max"] - prm[f"x{d}min"]) / prm[f"n{d}"]
        shifted = dict(prm, **{f"x{d}min": prm[f"x{d}min"] - 0.5 * dx, f"x{d}max": prm[f"x{d}max"] - 0.5 * dx})
        other = oracle.Grid(shifted)
        for name in ("gcov", "gcon", "gdet", "alpha"):
            assert np.allclose(grid.face[d][name], other.cent[name], rtol=1e-12, atol=1e-12), (d, name)


def test_cks_michel_data_at_zero_spin_is_radial():
    prm, P = problems.cks_bondi(8, 6, 5, a=0.0)
    grid = oracle.Grid(prm)
    st = oracle.fluid_state(P, grid.cent, prm["gam"])
    u = np.array(st["ucon"][1:])
    x = np.array([grid.x1c, grid.x2c, grid.x3c])
    cross = np.cross(u, x, axis=0)
    assert np.abs(cross).max() < 1e-12 * np.abs(u).max() * np.abs(x).max()
    assert (np.einsum("i...,i...->...", u, x) < 0).all()          # inflow
    B = P[5:8]
    assert np.abs(np.cross(B, x, axis=0)).max() < 1e-12 * np.abs(B).max() * np.abs(x).max()


def test_cks_stationary_flow_converges_at_second_order():
    it = (slice(None), slice(3, -3), slice(3, -3), slice(3, -3))
    err = {}
    for n, dt, ns in ((12, 0.3, 6), (24, 0.15, 12)):
        prm, P = problems.cks_bondi(n, n, n, a=0.0)
        grid = oracle.Grid(prm)
        assert dt < oracle.get_dt(P, grid)
        Q = P.copy()
        for _ in range(ns):
            Q, _, _ = oracle.step(Q, grid, dt)
        err[n] = np.abs(Q[it] - P[it]).mean(axis=(1, 2, 3))
    ratio = err[12] / err[24]
    total = err[12].sum() / err[24].sum()
    print("error 12^3", err[12], "24^3", err[24], "ratios", ratio, "total", total)
    assert total > 3.2
    assert (ratio[[0, 1, 5, 6, 7]] > 2.5).all()   # first order would give 2


def test_cks_rejects_a_window_of_x3_planes():
    prm, P = problems.cks_bondi(6, 5, 4)
    grid = oracle.Grid(prm)
    with pytest.raises(ValueError):
        oracle.substep(P[:, :8], P[:, 3:5, 3:-3, 3:-3], grid, 0.1, window=True)
