"""Pins of the oracle's point physics: four-vectors, fluxes, signal speeds,
reconstruction and the LLF flux, against closed forms and invariants."""

import numpy as np

import problems
from oracle import grid as G
from oracle.physics import fluid_state, flux, conserved, signal_speeds
from oracle.recon import mc_slope, weno5_edge, reconstruct


def kerr_geo(n=50, seed=0, rmin=1.2):
    """Random points of the torus geometry between r = rmin and r = 500."""
    prm, _ = problems.fm_torus(n1=16, n2=16, n3=1)
    rng = np.random.default_rng(seed)
    x1 = rng.uniform(np.log(rmin), np.log(500.0), n)
    x2 = rng.uniform(0.02, 0.98, n)
    return prm, G.metric(x1, x2, prm)


def random_prims(n, seed=1, vmax=2.0, bmax=2.0):
    rng = np.random.default_rng(seed)
    P = np.empty((8, n))
    P[0] = rng.uniform(0.1, 2.0, n)
    P[1] = rng.uniform(0.01, 2.0, n)
    P[2:5] = rng.uniform(-vmax, vmax, (3, n)) * np.array([[0.2], [0.05], [0.1]])
    P[5:8] = rng.uniform(-bmax, bmax, (3, n)) * np.array([[0.5], [0.1], [0.2]])
    return P


def physical_prims(geo, n, seed=1):
    """Random states with O(1) Lorentz factors and field in every geometry
    (code-coordinate components scaled by 1/sqrt(g_ii))."""
    P = random_prims(n, seed)
    for i in range(3):
        P[2 + i] /= np.sqrt(geo["gcov"][i + 1, i + 1])
        P[5 + i] /= np.sqrt(geo["gcov"][i + 1, i + 1])
    return P


def test_four_vector_invariants_kerr():
    prm, geo = kerr_geo()
    P = physical_prims(geo, 50)
    st = fluid_state(P, geo, prm["gam"])
    uu = sum(st["ucon"][m] * st["ucov"][m] for m in range(4))
    bu = sum(st["bcon"][m] * st["ucov"][m] for m in range(4))
    assert np.allclose(uu, -1.0, atol=1e-12)
    scale = np.sqrt(np.abs(st["bsq"])) * st["lorentz"]
    assert (np.abs(bu) < 1e-13 * scale * 1e2).all()
    for i in range(3):
        Bi = st["bcon"][i + 1] * st["ucon"][0] - st["bcon"][0] * st["ucon"][i + 1]
        assert np.allclose(Bi, P[5 + i], rtol=1e-10, atol=1e-12)


def test_flat_space_special_relativity_limits():
    """B = 0, flat space: U = (rho W, w W^2 - p - rho W... ) written out from SR hydro."""
    eta = np.diag([-1.0, 1, 1, 1])
    geo = dict(gcov=eta[:, :, None], gcon=eta[:, :, None], gdet=np.ones(1), alpha=np.ones(1))
    gam = 5.0 / 3.0
    v = np.array([0.3, -0.2, 0.1])
    lor = 1.0 / np.sqrt(1.0 - v @ v)
    P = np.array([1.3, 0.7, *(lor * v), 0.0, 0.0, 0.0])[:, None]
    st = fluid_state(P, geo, gam)
    U = conserved(st, geo["gdet"])[:, 0]
    p = (gam - 1) * 0.7
    w = 1.3 + 0.7 + p
    assert np.isclose(st["lorentz"][0], lor, rtol=1e-14)
    assert np.isclose(U[0], 1.3 * lor, rtol=1e-14)
    # T^t_t + rho u^t = -(w lor^2 - p) + rho lor
    assert np.isclose(U[1], -(w * lor * lor - p) + 1.3 * lor, rtol=1e-13)
    # T^t_i = w lor^2 v_i
    assert np.allclose(U[2:5], w * lor * lor * v, rtol=1e-13)
    F1 = flux(st, 1, geo["gdet"])[:, 0]
    assert np.isclose(F1[2], w * lor * lor * v[0] ** 2 + p, rtol=1e-13)
    assert np.isclose(F1[0], 1.3 * lor * v[0], rtol=1e-14)


def test_normal_b_flux_zero_and_conserved_b():
    prm, geo = kerr_geo()
    P = physical_prims(geo, 50)
    st = fluid_state(P, geo, prm["gam"])
    for d in (1, 2, 3):
        F = flux(st, d, geo["gdet"])
        assert (F[4 + d] == 0.0).all()
    U = conserved(st, geo["gdet"])
    assert np.array_equal(U[5:8], geo["gdet"] * P[5:8])


def _flat_geo(n):
    eta = np.diag([-1.0, 1, 1, 1])
    return dict(gcov=np.repeat(eta[:, :, None], n, 2), gcon=np.repeat(eta[:, :, None], n, 2),
                gdet=np.ones(n), alpha=np.ones(n))


def test_speeds_at_rest_and_boosted():
    gam = 4.0 / 3.0
    geo = _flat_geo(1)
    # at rest, no field: +-c_s
    P = np.array([1.0, 1.0, 0, 0, 0, 0, 0, 0.0])[:, None]
    st = fluid_state(P, geo, gam)
    cp, cm = signal_speeds(st, geo, 1, gam)
    cs = np.sqrt(gam * (gam - 1) / (1 + gam))
    assert np.isclose(cp[0], cs, rtol=1e-14) and np.isclose(cm[0], -cs, rtol=1e-14)
    # boosted along x1 with v = 0.5 and c_s = 0.5: relativistic addition -> 0.8 and 0
    # c_s^2 = gam p / w = 0.25  ->  u = rho * 0.25/(gam (gam-1) - 0.25 gam)
    rho = 1.0
    u = 0.25 * rho / (gam * (gam - 1.0) - 0.25 * gam)
    v = 0.5
    lor = 1 / np.sqrt(1 - v * v)
    P = np.array([rho, u, lor * v, 0, 0, 0, 0, 0.0])[:, None]
    st = fluid_state(P, geo, gam)
    cp, cm = signal_speeds(st, geo, 1, gam)
    assert np.isclose(cp[0], 0.8, rtol=1e-13) and abs(cm[0]) < 1e-13


def test_fast_speed_is_perpendicular_magnetosonic_root():
    """At rest, c^2 = v_A^2 + c_s^2 (1 - v_A^2) is the root of the fast/slow
    dispersion relation X^2 - [v_A^2 + c_s^2 (1 - v_A^2) + c_s^2 v_A^2 cos^2]X
    + c_s^2 v_A^2 cos^2 = 0 at 90 degrees, and bounds it at every angle."""
    gam = 4.0 / 3.0
    geo = _flat_geo(1)
    P = np.array([1.0, 1.0, 0, 0, 0, 0.0, 1.0, 0.0])[:, None]    # B perpendicular to x1
    st = fluid_state(P, geo, gam)
    cp, _ = signal_speeds(st, geo, 1, gam)
    va2 = 1.0 / (1.0 + 1.0 + gam * 1.0)
    cs2 = gam * (gam - 1.0) / (1.0 + gam)
    for cos2 in (0.0, 0.3, 1.0):
        bsum = va2 + cs2 * (1 - va2) + cs2 * va2 * cos2
        xfast = 0.5 * (bsum + np.sqrt(bsum * bsum - 4 * cs2 * va2 * cos2))
        if cos2 == 0.0:
            assert np.isclose(cp[0] ** 2, xfast, rtol=1e-14)
        assert cp[0] ** 2 >= xfast - 1e-15


def test_mc_slope_properties():
    x = np.linspace(-1, 1, 11)
    lin = 3.0 * x + 1.0
    s = mc_slope(lin[:-2], lin[1:-1], lin[2:])
    assert np.allclose(s, 3.0 * (x[1] - x[0]), rtol=1e-14)
    # extremum -> 0
    assert mc_slope(np.array(1.0), np.array(2.0), np.array(1.5)) == 0.0
    # limited by 2 |Delta-|
    assert mc_slope(np.array(0.0), np.array(0.1), np.array(5.0)) == 0.2
    L, R = reconstruct(lin[None, :], 1, 0, 2, 9)
    assert np.allclose(L, R, rtol=1e-14, atol=1e-14)
    assert np.allclose(L[0], 0.5 * (lin[1:8] + lin[2:9]), rtol=1e-13)


def test_weno5_exactness_and_order():
    rng = np.random.default_rng(3)
    for _ in range(20):
        c = rng.normal(size=3)
        q = lambda t: c[0] + c[1] * t + c[2] * t * t
        xs = q(np.arange(-2, 3.0))
        assert np.isclose(weno5_edge(*xs), q(0.5), rtol=1e-12, atol=1e-12)
        assert np.isclose(weno5_edge(*xs[::-1]), q(-0.5), rtol=1e-12, atol=1e-12)
    # linear data gives equal smoothness indicators, hence the linear weights, whose
    # combination is the degree-4 interpolant (3, -20, 90, 60, -5)/128
    cu = lambda t: 0.3 * t ** 3 - t * t + 2 * t - 1
    xs = np.arange(-2, 3.0) * 0.7 + 0.1
    lin = 2.0 * xs + 1
    assert np.isclose(weno5_edge(*lin), np.dot([3, -20, 90, 60, -5], lin) / 128, rtol=1e-14)
    # fifth order on smooth monotone data
    errs = []
    for h in (0.1, 0.05, 0.025):
        t = np.arange(-2, 3.0) * h
        errs.append(abs(weno5_edge(*np.exp(t)) - np.exp(0.5 * h)))
    rate = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
    assert min(rate) > 4.5


def test_reconstruction_mirror_symmetry():
    rng = np.random.default_rng(4)
    P = rng.normal(size=(1, 20))
    for recon in (0, 1):
        L, R = reconstruct(P, 1, recon, 3, 18)
        Lm, Rm = reconstruct(P[:, ::-1], 1, recon, 3, 18)
        # face f of the mirrored array is face 20 - f of the original, with L <-> R
        assert np.allclose(L[0], Rm[0][::-1], rtol=1e-14, atol=1e-15)
        assert np.allclose(R[0], Lm[0][::-1], rtol=1e-14, atol=1e-15)


def test_llf_consistency_uniform_state():
    """Identical left and right states give the physical flux exactly."""
    import oracle
    prm, P = problems.linear_modes(n=8)
    P[:, :] = np.array([1.0, 1.0, 0.1, -0.05, 0.02, 1.0, 0.3, -0.2])[:, None, None, None]
    g = oracle.Grid(prm)
    F, C = oracle.face_fluxes(P, g, 2)
    geo = _flat_geo(1)
    st = fluid_state(P[:, 4, 4, 4][:, None], geo, prm["gam"])
    exact = flux(st, 2, geo["gdet"])[:, 0]
    assert np.array_equal(F[:, 4, 4, 4], exact)
