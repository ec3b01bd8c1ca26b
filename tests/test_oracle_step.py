"""Pins of the oracle's full step: Flux-CT invariance, conservation, the Courant
step, convergence on the paper's test problems (Tests section), torus
equilibrium properties, bounds and fixup definitions, and the x3 window."""

import numpy as np
import pytest

import problems
import oracle
from oracle.step import flux_ct, fixup, floors, substep, fill_ghosts, _interior
from problems.modes import mode_solution

NG = 3


def interior(P, prm):
    return P[:, NG:NG + prm["n3"], NG:NG + prm["n2"], NG:NG + prm["n1"]]


def test_flux_ct_preserves_corner_divb_on_random_fluxes():
    prm, P = problems.linear_modes(n=8)
    rng = np.random.default_rng(11)
    g = oracle.Grid(prm)
    shape = P.shape
    F = [rng.normal(size=shape) for _ in range(3)]
    flux_ct(*F, g)
    B0 = rng.normal(size=P.shape)
    P[:] = B0
    dt = 0.1
    n = 8
    K = J = I = slice(NG, NG + n)
    Kp = Jp = Ip = slice(NG + 1, NG + n + 1)
    dx = g.dx
    P1 = P.copy()
    for b in (5, 6, 7):
        P1[b, K, J, I] = P[b, K, J, I] - dt * ((F[0][b, K, J, Ip] - F[0][b, K, J, I]) / dx[0]
                                               + (F[1][b, K, Jp, I] - F[1][b, K, J, I]) / dx[1]
                                               + (F[2][b, Kp, J, I] - F[2][b, K, J, I]) / dx[2])
    # divergence at the corners whose 8 cells are all updated (no wrap needed)
    def cdiv(Q):
        G = [Q[5 + d, K, J, I] for d in range(3)]
        d1 = G[0][1:, 1:, 1:] - G[0][1:, 1:, :-1] + G[0][:-1, 1:, 1:] - G[0][:-1, 1:, :-1] \
            + G[0][1:, :-1, 1:] - G[0][1:, :-1, :-1] + G[0][:-1, :-1, 1:] - G[0][:-1, :-1, :-1]
        d2 = G[1][1:, 1:, 1:] - G[1][1:, :-1, 1:] + G[1][:-1, 1:, 1:] - G[1][:-1, :-1, 1:] \
            + G[1][1:, 1:, :-1] - G[1][1:, :-1, :-1] + G[1][:-1, 1:, :-1] - G[1][:-1, :-1, :-1]
        d3 = G[2][1:, 1:, 1:] - G[2][:-1, 1:, 1:] + G[2][1:, :-1, 1:] - G[2][:-1, :-1, 1:] \
            + G[2][1:, 1:, :-1] - G[2][:-1, 1:, :-1] + G[2][1:, :-1, :-1] - G[2][:-1, :-1, :-1]
        return d1 / (4 * dx[0]) + d2 / (4 * dx[1]) + d3 / (4 * dx[2])
    change = cdiv(P1) - cdiv(P)
    assert np.abs(change).max() < 1e-12 * np.abs(cdiv(P)).max()


def test_uniform_state_preserved_flat():
    prm, P = problems.linear_modes(n=8)
    P[:, :] = np.array([1.0, 0.5, 0.2, -0.1, 0.05, 0.7, 0.3, -0.4])[:, None, None, None]
    g = oracle.Grid(prm)
    P1, _, info = oracle.step(P, g, 0.01)
    d = interior(P1, prm) - interior(P, prm)
    assert np.abs(d).max() < 1e-14
    assert info["fail_predictor"] == info["fail_corrector"] == 0


def test_courant_step_on_box_background():
    """Background rho = u = 1, B = x, gamma = 4/3: ctop = sqrt(c^2) = 0.658280589
    in every direction, so dt = 0.9 / (3 * 32 * 0.658280589) = 0.0142416473."""
    prm, P = problems.linear_modes(n=32)
    g = oracle.Grid(prm)
    dt = oracle.get_dt(P, g)
    assert abs(dt / 0.0142416473 - 1.0) < 1e-3
    P[:, :] = problems.modes.BACKGROUND[:, None, None, None]
    assert abs(oracle.get_dt(P, g) - 0.0142416473) < 1e-10


def test_periodic_box_conserves_totals_and_divb():
    prm, P = problems.linear_modes(n=12, amp=1e-2)
    g = oracle.Grid(prm)
    U0 = oracle.prim_to_cons(P, g).sum(axis=(1, 2, 3))
    dt = oracle.get_dt(P, g)
    for _ in range(4):
        P, dt, _ = oracle.step(P, g, dt)
    U1 = oracle.prim_to_cons(P, g).sum(axis=(1, 2, 3))
    # mass, energy, momenta and B totals are conserved up to the inversion's round-off
    assert np.allclose(U1, U0, rtol=0, atol=1e-11 * np.abs(U0).max())
    assert oracle.divb(P, g) < 1e-12


def _mode_error(n, T, recon=0, kvec=(1, 1, 0), n3=1):
    prm, P = problems.linear_modes(n=n, kvec=kvec, n3=n3, recon=recon)
    g = oracle.Grid(prm)
    t, dt = 0.0, oracle.get_dt(P, g)
    while t < T - 1e-14:
        dt = min(dt, T - t)
        P, dtn, _ = oracle.step(P, g, dt)
        t += dt
        dt = min(dtn, 1.3 * dt)
    return np.abs(interior(P, prm) - mode_solution(prm, T)).mean()


@pytest.mark.parametrize("recon", [0, 1])
def test_linear_modes_second_order(recon):
    """Tests section, linear modes: the L1 error against the analytic solution
    falls at second order (2D slice of the mode set, k = 2 pi (1, 1, 0))."""
    e = [_mode_error(n, 0.5, recon) for n in (16, 32, 64)]
    slopes = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert (slopes > 1.8).all() and (slopes < 2.4).all(), (e, slopes)


def test_linear_modes_3d_converge():
    e = [_mode_error(n, 0.25, 0, kvec=(1, 1, 1), n3=n) for n in (8, 16)]
    assert np.log2(e[0] / e[1]) > 1.7, e


def test_bondi_stationary_second_order():
    """Tests section, un-magnetised Bondi flow on a 2D N^2 grid: the deviation
    from the stationary solution (outside r = 2.5) converges at second order."""
    errs = []
    for n in (16, 32, 64):
        prm, P0 = problems.bondi(n1=n, n2=n, n3=1)
        g = oracle.Grid(prm)
        P, t, dt = P0.copy(), 0.0, oracle.get_dt(P0, g)
        while t < 5.0 - 1e-12:
            dt = min(dt, 5.0 - t)
            P, dtn, _ = oracle.step(P, g, dt)
            t += dt
            dt = min(dtn, 1.3 * dt)
        m = g.r[NG:NG + n, NG:NG + n] > 2.5
        errs.append(np.abs(interior(P, prm)[0, 0] - interior(P0, prm)[0, 0])[m].mean())
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert (slopes > 1.8).all(), (errs, slopes)


def test_michel_constants_hold():
    from problems.bondi import michel_constants, michel_temperature
    n, tc, c1, c2 = michel_constants(8.0, 4.0 / 3.0)
    r = np.array([1.5, 3.0, 7.9, 8.0, 8.1, 20.0, 40.0])
    T = michel_temperature(r, 8.0, 4.0 / 3.0)
    ur = c1 / (r * r * T ** n)
    lhs = (1 + (n + 1) * T) ** 2 * (1 - 2 / r + ur * ur)
    assert np.allclose(lhs, c2, rtol=1e-12)
    assert np.allclose(r * r * T ** n * ur, c1, rtol=1e-14)


def test_torus_initial_data_pins():
    from problems.torus import fm_lnh, circular_orbit_ell
    a = 0.9375
    ell = circular_orbit_ell(12.0, a)
    assert abs(ell - 4.2812844685) < 1e-9
    h = 1e-4
    dl = (fm_lnh(np.array(12 + h), np.array(np.pi / 2), a, ell, 6.0)
          - fm_lnh(np.array(12 - h), np.array(np.pi / 2), a, ell, 6.0)) / (2 * h)
    assert abs(dl) < 1e-8
    assert fm_lnh(np.array(6.0), np.array(np.pi / 2), a, ell, 6.0) == 0.0
    # outer edge of the equatorial cross-section near r = 42
    rr = np.linspace(20, 60, 4001)
    lnh = fm_lnh(rr, np.full_like(rr, np.pi / 2), a, ell, 6.0)
    edge = rr[np.nonzero(lnh > 0)[0].max()]
    assert 40 < edge < 44
    prm, P = problems.fm_torus(n1=64, n2=48, n3=4)
    g = oracle.Grid(prm)
    Pi = interior(P, prm)
    assert Pi[0].max() == 1.0
    assert oracle.divb(P, g) < 1e-12
    # beta = max p_gas / max p_mag = 100 after scaling (b^2 in code coordinates)
    from oracle.physics import fluid_state
    geo = {k: v[..., NG:NG + 48, NG:NG + 64] for k, v in g.cent.items()}
    P0 = Pi.copy()
    P0[1] = problems.fm_torus(n1=64, n2=48, n3=4, noise=0.0)[1][1, NG:NG + 4, NG:NG + 48, NG:NG + 64]
    st = fluid_state(P0, geo, prm["gam"])
    beta = ((prm["gam"] - 1) * P0[1]).max() / (0.5 * st["bsq"]).max()
    assert abs(beta / 100.0 - 1.0) < 1e-10
    # inside the torus u/rho = (h - 1)/gamma (0.011768 at the pressure maximum)
    lmax = fm_lnh(np.array(12.0), np.array(np.pi / 2), a, ell, 6.0)
    assert abs(np.expm1(lmax) / prm["gam"] - 0.011768) < 1e-6
    body = P0[0] > 0.05
    x1c = prm["x1min"] + (np.arange(64) + 0.5) * g.dx[0]
    x2c = (np.arange(48) + 0.5) * g.dx[1]
    X1, X2 = np.meshgrid(x1c, x2c)
    th = oracle.grid.theta_of(X1, X2, prm)[0]
    lnh = fm_lnh(np.exp(X1), th, a, ell, 6.0)
    ratio = np.broadcast_to(np.expm1(lnh) / prm["gam"], P0[0].shape)
    assert np.allclose((P0[1] / P0[0])[body], ratio[body], rtol=1e-12)


def _torus_body_drift(n, T):
    """Relative L1 change of rho in the body of an unmagnetised, unperturbed
    Fishbone-Moncrief torus (rho > 0.1) after time T, on an n x n x 1 grid."""
    prm, P0 = problems.fm_torus(n1=n, n2=n, n3=1, noise=0.0, beta=float("inf"))
    assert np.abs(P0[5:]).max() == 0.0
    g = oracle.Grid(prm)
    P, t, dt = P0.copy(), 0.0, oracle.get_dt(P0, g)
    while t < T - 1e-12:
        dt = min(dt, T - t)
        P, dn, _ = oracle.step(P, g, dt)
        t += dt
        dt = min(dn, 1.3 * dt)
    r0 = P0[0, NG, NG:NG + n, NG:NG + n]
    r1 = P[0, NG, NG:NG + n, NG:NG + n]
    body = r0 > 0.1
    return np.abs(r1 - r0)[body].mean() / r0[body].mean()


def test_unmagnetised_torus_is_stationary():
    # the Fishbone-Moncrief torus is an equilibrium: without field and noise
    # its body drifts only by the truncation error, which falls at second order
    d = [_torus_body_drift(n, 3.0) for n in (32, 64)]
    assert d[1] < 2e-3 and np.log2(d[0] / d[1]) > 1.7, d


def test_floors_idempotent_monotone_and_noop_on_box():
    prm, P = problems.fm_torus(n1=32, n2=24, n3=2)
    g = oracle.Grid(prm)
    geo = {k: v[..., NG:NG + 24, NG:NG + 32] for k, v in g.cent.items()}
    rng = np.random.default_rng(12)
    Q = interior(P, prm).copy()
    Q[0] *= 10.0 ** rng.uniform(-8, 0, Q[0].shape)
    Q[1] *= 10.0 ** rng.uniform(-8, 2, Q[1].shape)
    Q[2:5] += rng.normal(size=Q[2:5].shape) * 3.0
    r = g.r[NG:NG + 24, NG:NG + 32]
    A = floors(Q.copy(), geo, r, prm)
    assert (A[0] >= Q[0]).all() and (A[1] >= Q[1]).all()
    B = floors(A.copy(), geo, r, prm)
    # a second pass may re-trim Gamma by one ulp, which b^2 amplifies by ~Gamma^2
    assert np.allclose(B, A, rtol=1e-11, atol=0)
    from oracle.physics import fluid_state
    st = fluid_state(A, geo, prm["gam"])
    assert (st["lorentz"] <= 50.0 * (1 + 1e-12)).all()
    assert (st["bsq"] / A[0] <= 400 * (1 + 1e-12)).all()
    assert (A[1] / A[0] <= 100 * (1 + 1e-12)).all()
    # the box background is far from every bound
    pb, Pb = problems.linear_modes(n=4)
    gb = oracle.Grid(pb)
    geob = {k: v[..., NG:NG + 4, NG:NG + 4] for k, v in gb.cent.items()}
    Qb = interior(Pb, pb).copy()
    assert np.array_equal(floors(Qb.copy(), geob, np.full((4, 4), 1e3), pb), Qb)


def test_fixup_matches_loop_in_any_order():
    rng = np.random.default_rng(13)
    P = rng.normal(size=(8, 5, 6, 7))
    failed = rng.random((5, 6, 7)) < 0.3
    ref = P.copy()
    idx = list(zip(*np.nonzero(failed)))
    rng.shuffle(idx)
    for (k, j, i) in idx:                 # plain loops, shuffled traversal
        acc = np.zeros(5)
        c = 0
        for dk in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    kk, jj, ii = k + dk, j + dj, i + di
                    if (dk, dj, di) == (0, 0, 0) or not (0 <= kk < 5 and 0 <= jj < 6 and 0 <= ii < 7):
                        continue
                    if not failed[kk, jj, ii]:
                        acc += P[:5, kk, jj, ii]
                        c += 1
        if c:
            ref[:5, k, j, i] = acc / c
    got = fixup(P.copy(), failed)
    assert np.allclose(got, ref, rtol=1e-14, atol=1e-15)
    assert np.array_equal(got[5:], P[5:])


def test_polar_reflection_is_involution():
    prm, P = problems.fm_torus(n1=16, n2=12, n3=4)
    g = oracle.Grid(prm)
    A = fill_ghosts(P.copy(), g)
    B = fill_ghosts(A.copy(), g)
    assert np.array_equal(A, B)
    # ghost row -1 mirrors row 0 with u~2 and B2 negated
    assert np.array_equal(A[3, :, NG - 1, :], -A[3, :, NG, :])
    assert np.array_equal(A[0, :, NG - 2, :], A[0, :, NG + 1, :])


def test_torus_divb_stays_roundoff_over_steps():
    prm, P = problems.fm_torus(n1=32, n2=24, n3=4)
    g = oracle.Grid(prm)
    dt = oracle.get_dt(P, g)
    for _ in range(5):
        P, dt, _ = oracle.step(P, g, dt)
    assert oracle.divb(P, g) < 1e-12


def test_window_step_equals_full_step():
    prm, P = problems.fm_torus(n1=24, n2=16, n3=24)
    g = oracle.Grid(prm)
    dt = oracle.get_dt(P, g)
    full, _, _ = oracle.step(P, g, dt)
    win = oracle.step_window(P, g, dt, 10, 12)
    ref = interior(full, prm)[:, 10:12]
    assert np.array_equal(win, ref)
    win0 = oracle.step_window(P, g, dt, 0, 1)     # wraps around the periodic x3 edge
    assert np.array_equal(win0, interior(full, prm)[:, 0:1])


def test_fixup_wraps_periodic_directions():
    """Across a periodic direction the neighbours of a failed zone are the
    zones on the other side of the seam: a brute-force loop with modular
    indices, and invariance under shifts of the seam (np.roll)."""
    rng = np.random.default_rng(17)
    P = rng.normal(size=(8, 5, 6, 7))
    failed = rng.random((5, 6, 7)) < 0.25
    failed[0, 0, 0] = failed[4, 5, 6] = True           # corners touch three seams
    for wrap in ((True, True, True), (True, False, True), (False, True, False)):
        ref = P.copy()
        for (k, j, i) in zip(*np.nonzero(failed)):
            acc, c = np.zeros(5), 0
            for dk in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    for di in (-1, 0, 1):
                        if (dk, dj, di) == (0, 0, 0):
                            continue
                        idx = []
                        for x, dx, n, w in ((k, dk, 5, wrap[0]), (j, dj, 6, wrap[1]), (i, di, 7, wrap[2])):
                            y = x + dx
                            if w:
                                y %= n
                            elif not 0 <= y < n:
                                y = None
                            idx.append(y)
                        if None in idx or failed[tuple(idx)]:
                            continue
                        acc += P[(slice(0, 5),) + tuple(idx)]
                        c += 1
            if c:
                ref[:5, k, j, i] = acc / c
        got = fixup(P.copy(), failed, wrap)
        assert np.allclose(got, ref, rtol=1e-14, atol=1e-15), wrap
    # seam placement does not matter where everything is periodic
    full = (True, True, True)
    base = fixup(P.copy(), failed, full)
    for shift in ((2, 0, 0), (0, 3, 0), (0, 0, 5), (1, 2, 3)):
        rolled = fixup(np.roll(P, shift, axis=(1, 2, 3)), np.roll(failed, shift, axis=(0, 1, 2)), full)
        assert np.array_equal(np.roll(rolled, [-s for s in shift], axis=(1, 2, 3)), base), shift


def test_step_with_a_failed_zone_at_the_seam_is_translation_invariant():
    """On a periodic box a zone whose inversion fails next to the x3 seam is
    repaired from the zones across the seam: rolling the initial state along
    x3 rolls the result. A cold zone moving at Lorentz factor ~ 40 into gas at
    rest makes the inversions around it fail in the corrector."""
    prm, P0 = problems.linear_modes(n=8)
    g = oracle.Grid(prm)
    Q = P0.copy()
    Q[1, NG, NG + 3, NG + 3] = 1e-6
    Q[2, NG, NG + 3, NG + 3] = 40.0
    dt = oracle.get_dt(Q, g)
    a, _, info = oracle.step(Q, g, dt)
    assert info["fail_predictor"] + info["fail_corrector"] > 0
    for s in (1, 3):
        R = Q.copy()
        R[:, NG:NG + 8] = np.roll(Q[:, NG:NG + 8], s, axis=1)
        b, _, _ = oracle.step(R, g, dt)
        bi = np.roll(interior(b, prm), -s, axis=1)
        assert np.allclose(bi, interior(a, prm), rtol=1e-12, atol=1e-14), s


def test_no_mass_enters_through_the_radial_outflow_faces():
    """The rest-mass flux through the inner radial face is never positive and
    through the outer one never negative: against the same faces computed
    without the outflow rule (Dirichlet x1 on the same filled state), the two
    boundary faces are min(F, 0) and max(F, 0) and every other face and
    component is unchanged. The grid starts at r = 3, outside the horizon,
    and the state streams into the domain at both ends so that the clip acts
    on both faces."""
    import math
    from oracle.step import face_fluxes
    prm, P = problems.fm_torus(n1=24, n2=12, n3=2)
    prm = dict(prm, x1min=math.log(3.0))
    g = oracle.Grid(prm)
    Q = P.copy()
    Q[2, :, :, NG:NG + 2] = 3.0
    Q[2, :, :, NG + 22:NG + 24] = -3.0
    Q = fill_ghosts(Q, g)
    F, _ = face_fluxes(Q, g, 1)
    prm_d = dict(prm, bc=[[problems.BC_DIRICHLET, problems.BC_DIRICHLET], prm["bc"][1], prm["bc"][2]])
    F0, _ = face_fluxes(Q, oracle.Grid(prm_d), 1)
    K, J = slice(NG, NG + 2), slice(NG, NG + 12)
    lo, hi = F0[0, K, J, NG], F0[0, K, J, NG + 24]
    assert np.any(lo > 0.0) and np.any(hi < 0.0)            # the rule has something to do
    assert np.array_equal(F[0, K, J, NG], np.minimum(lo, 0.0))
    assert np.array_equal(F[0, K, J, NG + 24], np.maximum(hi, 0.0))
    same = np.isfinite(F0)
    same[0, :, :, NG] = same[0, :, :, NG + 24] = False
    assert np.array_equal(F[same], F0[same])
