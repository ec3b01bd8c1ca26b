"""Pins of the oracle's 1D_W inversion: round trips, an independent root finder,
the root's defining equation, and failure detection."""

import numpy as np

import problems
from oracle import grid as G
from oracle.physics import fluid_state, conserved
from oracle.invert import invert, _prepare, V2MAX

from test_oracle_physics import kerr_geo, physical_prims, _flat_geo


def test_round_trip_kerr():
    prm, geo = kerr_geo(200, seed=5)
    P = physical_prims(geo, 200, seed=6)
    U = conserved(fluid_state(P, geo, prm["gam"]), geo["gdet"])
    guess = P.copy()
    guess[0] *= 1.3
    guess[1] *= 0.6
    guess[2:5] *= 0.8
    Q, failed = invert(U, guess, geo, prm["gam"])
    assert not failed.any()
    assert np.allclose(Q[0], P[0], rtol=1e-12)
    assert np.allclose(Q[1], P[1], rtol=1e-11)
    for i in range(3):
        sc = np.abs(P[2 + i]).max()
        assert np.allclose(Q[2 + i], P[2 + i], rtol=1e-11, atol=1e-12 * sc)
    assert np.array_equal(Q[5:8], U[5:8] / geo["gdet"])


def test_round_trip_cold_slow_flat():
    """u << rho and v << 1, where a naive W formulation cancels."""
    n = 100
    geo = _flat_geo(n)
    rng = np.random.default_rng(7)
    P = np.zeros((8, n))
    P[0] = 1.0
    P[1] = 10.0 ** rng.uniform(-9, -3, n)
    P[2:5] = rng.uniform(-1, 1, (3, n)) * 1e-5
    P[5:8] = rng.uniform(-1, 1, (3, n)) * 1e-2
    U = conserved(fluid_state(P, geo, 5.0 / 3.0), geo["gdet"])
    Q, failed = invert(U, np.broadcast_to(P[:, :1], P.shape).copy(), geo, 5.0 / 3.0)
    assert not failed.any()
    assert np.allclose(Q[1], P[1], rtol=1e-7)
    assert np.allclose(Q[2:5], P[2:5], rtol=1e-9, atol=1e-18)


def _f(W, D, qn_d, qtsq, qdb, bsq, gam):
    """The energy equation written from its definition, without the W' rewriting."""
    v2 = (qtsq * W * W + qdb * qdb * (bsq + 2 * W)) / ((bsq + W) ** 2 * W * W)
    p = (gam - 1) / gam * (W * (1 - v2) - D * np.sqrt(1 - v2))
    qn = qn_d - D
    return qn + W - p + 0.5 * bsq * (1 + v2) - 0.5 * qdb * qdb / (W * W)


def test_root_matches_bisection_and_definition():
    prm, geo = kerr_geo(30, seed=8)
    gam = prm["gam"]
    P = physical_prims(geo, 30, seed=9)
    st = fluid_state(P, geo, gam)
    U = conserved(st, geo["gdet"])
    Ut, D, Bn, qn_d, qtil, qtsq, qdb, bsq = _prepare(U, geo)
    # W from the true primitives satisfies f(W) = 0
    w_true = (P[0] + gam * P[1]) * st["lorentz"] ** 2
    fval = _f(w_true, D, qn_d, qtsq, qdb, bsq, gam)
    assert np.abs(fval).max() < 1e-10 * np.abs(w_true).max()
    # independent bisection on f over the physical interval finds the same W
    Q, failed = invert(U, P, geo, gam)
    for z in range(30):
        args = (D[z], qn_d[z], qtsq[z], qdb[z], bsq[z], gam)
        lo = D[z] * 1.0000001
        hi = 10.0 * w_true[z]
        while _f(hi, *args) < 0:
            hi *= 2
        # v^2 < 1 on the bracket's low end is needed for p; move up until valid
        while ((qtsq[z] * lo * lo + qdb[z] ** 2 * (bsq[z] + 2 * lo)) / ((bsq[z] + lo) ** 2 * lo * lo)) >= 1:
            lo *= 1.01
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if _f(mid, *args) > 0:
                hi = mid
            else:
                lo = mid
        w_bis = 0.5 * (lo + hi)
        lor = 1.0 / np.sqrt(1.0 - (qtsq[z] * w_bis ** 2 + qdb[z] ** 2 * (bsq[z] + 2 * w_bis))
                            / ((bsq[z] + w_bis) ** 2 * w_bis ** 2))
        assert abs(D[z] / lor - Q[0][z]) < 1e-9 * Q[0][z]
        assert abs(w_bis - w_true[z]) < 1e-9 * w_true[z]


def test_unmagnetised_flat_reduces_to_sr_hydro():
    n = 20
    geo = _flat_geo(n)
    rng = np.random.default_rng(10)
    gam = 4.0 / 3.0
    v = rng.uniform(-0.5, 0.5, (3, n))
    lor = 1 / np.sqrt(1 - (v * v).sum(0))
    rho = rng.uniform(0.5, 2, n)
    u = rng.uniform(0.1, 2, n)
    p = (gam - 1) * u
    w = rho + u + p
    # SR hydro conserved variables written out directly
    U = np.zeros((8, n))
    U[0] = rho * lor
    U[1] = -(w * lor * lor - p) + rho * lor
    U[2:5] = w * lor * lor * v
    Q, failed = invert(U, np.broadcast_to(np.array([1, 1, 0, 0, 0, 0, 0, 0.0])[:, None], (8, n)).copy(),
                       geo, gam)
    assert not failed.any()
    assert np.allclose(Q[0], rho, rtol=1e-12) and np.allclose(Q[1], u, rtol=1e-11)
    assert np.allclose(Q[2:5], lor * v, rtol=1e-11, atol=1e-13)


def test_failures_flagged_and_guess_kept():
    geo = _flat_geo(3)
    gam = 4.0 / 3.0
    P = np.array([[1.0, 1.0, 0.1, 0, 0, 0.5, 0, 0]] * 3).T
    U = conserved(fluid_state(P, geo, gam), geo["gdet"])
    U[1, 0] = 50.0            # energy far above rest mass + momentum: no physical root
    U[2, 1] = 1e3             # momentum far beyond the energy: superluminal
    U[0, 2] = np.nan
    guess = P.copy()
    Q, failed = invert(U, guess, geo, gam)
    assert failed.all()
    assert np.array_equal(Q[:5], guess[:5])
