"""Pins of the oracle's coordinates, metric and connection against closed forms."""

import numpy as np
import pytest

import problems
from oracle import grid as G


def torus_prm():
    prm, _ = problems.fm_torus(n1=16, n2=16, n3=1)
    return prm


def test_fmks_theta_endpoints_and_monotone():
    prm = torus_prm()
    for x1 in (prm["x1min"], 0.0, np.log(1000.0)):
        th0, _, _ = G.theta_of(np.float64(x1), np.float64(0.0), prm)
        thh, _, _ = G.theta_of(np.float64(x1), np.float64(0.5), prm)
        th1, _, _ = G.theta_of(np.float64(x1), np.float64(1.0), prm)
        assert abs(th0) < 1e-15 and abs(thh - np.pi / 2) < 1e-15 and abs(th1 - np.pi) < 1e-15
    x1, x2 = np.meshgrid(np.linspace(prm["x1min"], np.log(1000), 40), np.linspace(0, 1, 401))
    _, _, dth2 = G.theta_of(x1, x2, prm)
    assert (dth2 > 0).all()
    # derivatives of the map agree with centred differences
    th, d1, d2 = G.theta_of(x1, x2, prm)
    h = 1e-6
    n1 = (G.theta_of(x1 + h, x2, prm)[0] - G.theta_of(x1 - h, x2, prm)[0]) / (2 * h)
    n2 = (G.theta_of(x1, x2 + h, prm)[0] - G.theta_of(x1, x2 - h, prm)[0]) / (2 * h)
    assert np.allclose(d1, n1, atol=1e-8) and np.allclose(d2, n2, atol=1e-7)


def test_mks_theta_map():
    # plain MKS: theta(0) = 0, theta(1/2) = pi/2, theta(1) = pi, mirror symmetry
    # about the equator, monotone for 0 < h <= 1, independent of x1; h = 1 is
    # the uniform map theta = pi x2 of exponential Kerr-Schild coordinates
    prm = problems.fm_torus(n1=16, n2=16, n3=1, coords=problems.KERR_MKS)[0]
    assert prm["coords"] == problems.KERR_MKS and prm["hslope"] == 0.3
    x2 = np.linspace(0.0, 1.0, 1001)
    for x1 in (prm["x1min"], 2.0):
        th, d1, d2 = G.theta_of(np.full_like(x2, x1), x2, prm)
        assert abs(th[0]) < 1e-15 and abs(th[500] - np.pi / 2) < 1e-15 and abs(th[-1] - np.pi) < 1e-15
        assert np.allclose(th + th[::-1], np.pi, atol=1e-14)
        assert (np.diff(th) > 0).all() and (d1 == 0).all()
        h = 1e-6
        num = (G.theta_of(np.full_like(x2, x1), x2 + h, prm)[0] - G.theta_of(np.full_like(x2, x1), x2 - h, prm)[0]) / (2 * h)
        assert np.allclose(d2, num, atol=1e-7)
    # d theta / d x2 is (2 - h) pi at the poles and h pi at the equator: MKS
    # concentrates zones toward the equator
    assert d2[0] / d2[500] == pytest.approx((2.0 - 0.3) / 0.3, rel=1e-12)
    ks = dict(prm, hslope=1.0)
    th, _, d2 = G.theta_of(np.full_like(x2, 1.0), x2, ks)
    assert np.allclose(th, np.pi * x2, rtol=0, atol=4e-16) and np.allclose(d2, np.pi, rtol=1e-15)


def test_horizon_rule():
    prm = torus_prm()
    a = prm["a"]
    rhor = 1 + np.sqrt(1 - a * a)
    dx1 = (prm["x1max"] - prm["x1min"]) / prm["n1"]
    assert abs((np.log(rhor) - prm["x1min"]) / dx1 - 5.5) < 1e-12
    big = problems.fm_torus(n1=288, n2=8, n3=1)[0]
    assert abs(np.exp(big["x1min"]) - 1.18523075) < 1e-8
    assert abs((big["x1max"] - big["x1min"]) / 288 - 0.0233952007) < 1e-10


def test_kerr_inverse_and_determinant_closed_forms():
    """g^{mu nu} and sqrt(-g) in code coordinates match the Kerr-Schild closed
    forms transformed with the inverse Jacobian."""
    prm = torus_prm()
    a = prm["a"]
    x1, x2 = np.meshgrid(np.linspace(prm["x1min"], np.log(1000), 7), np.linspace(0.05, 0.95, 9))
    m = G.metric(x1, x2, prm)
    r = np.exp(x1)
    th, d1, d2 = G.theta_of(x1, x2, prm)
    s, c = np.sin(th), np.cos(th)
    sig = r * r + a * a * c * c
    dl = r * r - 2 * r + a * a
    gks = np.zeros((4, 4) + r.shape)
    gks[0, 0] = -(1 + 2 * r / sig)
    gks[0, 1] = gks[1, 0] = 2 * r / sig
    gks[1, 1] = dl / sig
    gks[1, 3] = gks[3, 1] = a / sig
    gks[2, 2] = 1 / sig
    gks[3, 3] = 1 / (sig * s * s)
    Ji = np.zeros((4, 4) + r.shape)       # dX^mu / dx_KS^a
    Ji[0, 0] = 1
    Ji[1, 1] = 1 / r
    Ji[2, 1] = -d1 / (d2 * r)
    Ji[2, 2] = 1 / d2
    Ji[3, 3] = 1
    gcon = np.einsum("ma...,ab...,nb...->mn...", Ji, gks, Ji)
    # the code-coordinate metric is badly scaled (g_11 ~ r^2 at r ~ 1000), so compare
    # each component on the scale sqrt(|g^mm g^nn|) of its row and column
    diag = np.abs(np.array([gcon[i, i] for i in range(4)]))
    scale = np.sqrt(diag[:, None] * diag[None, :])
    assert (np.abs(m["gcon"] - gcon) <= 1e-11 * scale).all()
    assert np.allclose(m["gdet"], sig * s * r * d2, rtol=1e-12)
    ident = np.einsum("ab...,bc...->ac...", m["gcov"], m["gcon"])
    assert np.allclose(ident, np.eye(4)[:, :, None, None], atol=1e-11)
    assert np.allclose(m["alpha"], 1 / np.sqrt(1 + 2 * r / sig), rtol=1e-13)


def test_minkowski_geometry_exact():
    prm, _ = problems.linear_modes(n=8)
    g = G.Grid(prm)
    assert (g.cent["gcov"][:, :, 3, 3] == np.diag([-1.0, 1, 1, 1])).all()
    assert (g.cent["gdet"] == 1.0).all() and (g.conn == 0.0).all()


def _gcov_cs(x1, x2, prm, d, h=1e-30):
    """Complex-step derivative of g_code along x1 (d=1) or x2 (d=2)."""
    z1 = x1 + (1j * h if d == 1 else 0)
    z2 = x2 + (1j * h if d == 2 else 0)
    return np.imag(G.gcov_code(z1, z2, prm)) / h


def test_connection_metric_compatibility():
    """nabla_l g_mn = d_l g_mn - Gamma^k_lm g_kn - Gamma^k_ln g_mk = 0, with d_l
    g taken by complex step (independent of the finite difference)."""
    prm = torus_prm()
    x1, x2 = np.meshgrid(np.linspace(prm["x1min"] + 0.3, np.log(800), 5), np.linspace(0.1, 0.9, 5))
    gam = G.connection(x1, x2, prm)
    gc = G.gcov_code(x1, x2, prm)
    assert np.array_equal(gam, np.swapaxes(gam, 1, 2))
    dg = np.zeros((4, 4, 4) + x1.shape)
    dg[1] = _gcov_cs(x1, x2, prm, 1)
    dg[2] = _gcov_cs(x1, x2, prm, 2)
    cov = dg - np.einsum("klm...,kn...->lmn...", gam, gc) - np.einsum("kln...,mk...->lmn...", gam, gc)
    scale = np.abs(dg).max()
    assert np.abs(cov).max() < 2e-8 * scale
