"""Pins of the electron-heating oracle (readings E1-E6 in oracle/electrons.py)
against properties fixed by the equations: the primitives' own ghost rules,
exact transport of a passive scalar by a uniform flow (second-order
convergence), conservation of a uniform scalar, the scale invariance of ideal
MHD, a proportional-partition invariant, the bounds, and the published limits
of the heating models."""

import numpy as np
import pytest

import oracle
import problems
from oracle import electrons as el
from problems.params import base_problem, NG, BC_DIRICHLET


def _interior(prm):
    return (slice(None), slice(NG, NG + prm["n3"]), slice(NG, NG + prm["n2"]), slice(NG, NG + prm["n1"]))


def _evolve(prm, P, E, nsteps, dt=None, model=el.MODEL_CONSTANT, fel=0.5):
    """nsteps steps at the fixed step dt, or at the Courant step when dt is None."""
    g = oracle.Grid(prm)
    adapt = dt is None
    if adapt:
        dt = oracle.get_dt(P, g)
    for _ in range(nsteps):
        P, E, dn = el.step(P, E, g, dt, model, fel)
        if adapt:
            dt = min(dn, 1.3 * dt)
    return P, E


@pytest.mark.parametrize("make", [
    lambda: problems.fm_torus(n1=24, n2=12, n3=4),
    lambda: problems.bondi(n1=16, n2=8, n3=2, a=0.5),
    lambda: problems.linear_modes(n=8, n3=5),
], ids=["torus_polar_outflow", "bondi", "periodic"])
def test_scalar_ghosts_follow_the_primitive_rules(make):
    # E1: a scalar's ghosts are those of a primitive that no boundary rule
    # changes (rho and u: no sign flip on the axis, no inflow fix)
    prm, _ = make()
    rng = np.random.default_rng(5)
    shape = problems.params.padded_shape(prm)
    P = rng.random(shape) * 0.1
    P[2:5] *= 0.01
    E = rng.random(shape[1:])[None].repeat(2, axis=0)
    E[1] = rng.random(shape[1:])
    P[0], P[1] = E[0], E[1]
    g = oracle.Grid(prm)
    oracle.fill_ghosts(P, g)
    el.fill_scalar_ghosts(E, g)
    assert np.array_equal(E[0], P[0]) and np.array_equal(E[1], P[1])


def test_dirichlet_scalar_ghosts_are_kept():
    prm, _ = problems.linear_modes(n=8, n3=4)
    prm["bc"] = [[BC_DIRICHLET, BC_DIRICHLET]] * 3
    E = np.random.default_rng(1).random((2,) + problems.params.padded_shape(prm)[1:])
    assert np.array_equal(el.fill_scalar_ghosts(E.copy(), oracle.Grid(prm)), E)


def _uniform_flow(n, v1=0.5):
    """rho = 1, u = 0.1, u~1 = v1, B = 0 (Minkowski, periodic): the fluid is an
    exact stationary solution, and K_e rides on it as a passive scalar."""
    prm = base_problem(n, 2, 2, gam=5.0 / 3.0, x2max=2.0 / n, x3max=2.0 / n)
    P = np.zeros(problems.params.padded_shape(prm))
    P[0], P[1], P[2] = 1.0, 0.1, v1
    x = (np.arange(n) + 0.5) / n
    E = problems.electron_scalars(P, prm["gam"])
    E[1, :, :, NG:NG + n] = 0.03 * (1.0 + 0.5 * np.sin(2.0 * np.pi * x))
    return prm, P, E, x


def test_uniform_flow_transports_the_electron_entropy():
    # E2/E3: d(rho u^t K)/dt + d(rho u^1 K)/dx = 0 with rho, u^mu constant is
    # translation at u^1/u^t; the MC scheme converges at second order
    errs = []
    for n in (32, 64):
        prm, P, E, x = _uniform_flow(n)
        P1, E1 = _evolve(prm, P, E, n, dt=0.25 / n)
        t = 0.25
        v = 0.5 / np.sqrt(1.25)
        exact = 0.03 * (1.0 + 0.5 * np.sin(2.0 * np.pi * (x - v * t)))
        it = _interior(prm)
        np.testing.assert_allclose(P1[it], P[it], rtol=1e-12, atol=1e-14)   # the fluid does not change
        assert np.ptp(E1[0][it[1:]]) < 1e-13                               # nor its entropy
        errs.append(np.mean(np.abs(E1[1, NG, NG, NG:NG + n] - exact)))
    assert errs[1] < 2e-5
    assert errs[0] / errs[1] > 3.3, errs


def test_uniform_scalar_stays_uniform_in_a_magnetised_flow():
    # E3: with K uniform, U_K(n+1) = K (D_base - dt div F_mass) = K D(n+1) (the
    # mass equation), so without heating (f_e = 0) K_e stays exactly uniform;
    # E4 is inactive here and the primitives are the plain step's
    prm, P = problems.linear_modes(n=12, n3=4, amp=1e-3)
    it = _interior(prm)
    E = problems.electron_scalars(P, prm["gam"])
    E[1] = 0.25 * np.min(E[1][it[1:]])
    g = oracle.Grid(prm)
    dt = oracle.get_dt(P, g)
    Pa, Ea = P, E
    Pb = P
    for _ in range(3):
        Pa, Ea, _ = el.step(Pa, Ea, g, dt, el.MODEL_CONSTANT, 0.0)
        Pb = oracle.step(Pb, g, dt)[0]
    assert np.array_equal(Pa[it], Pb[it])
    k0 = E[1, NG, NG, NG]
    assert np.max(np.abs(Ea[1][it[1:]] / k0 - 1.0)) < 1e-13


def _sod(n, lam=1.0, gam=5.0 / 3.0, b=0.3):
    """A periodic magnetised shock tube with every density scaled by lam."""
    prm = base_problem(n, 2, 2, gam=gam, x2max=2.0 / n, x3max=2.0 / n)
    P = np.zeros(problems.params.padded_shape(prm))
    x = (np.arange(n) + 0.5) / n
    hi = (x > 0.25) & (x < 0.75)
    P[0, :, :, NG:NG + n] = lam * np.where(hi, 1.0, 0.125)
    P[1, :, :, NG:NG + n] = lam * np.where(hi, 1.0, 0.1)
    P[5, :, :, NG:NG + n] = np.sqrt(lam) * b
    P[6, :, :, NG:NG + n] = np.sqrt(lam) * 0.5 * b
    return prm, P


@pytest.mark.parametrize("model", [el.MODEL_CONSTANT, el.MODEL_KAWAZURA, el.MODEL_WERNER,
                                   el.MODEL_ROWAN, el.MODEL_HOWES, el.MODEL_SHARMA])
def test_scale_invariance(model):
    # ideal MHD has no density scale: rho, u -> lam rho, lam u and B -> sqrt(lam) B
    # map solutions to solutions, so K_tot -> lam^(1-gamma) K_tot and
    # K_e -> lam^(1-gamma_e) K_e. Shocks heat strongly here, so this fixes the
    # rho^(gamma - gamma_e) factor of E5 and the scale-free arguments of E6.
    n, lam = 48, 8.0
    out = []
    for s in (1.0, lam):
        prm, P = _sod(n, s)
        E = problems.electron_scalars(P, prm["gam"], te_ti=0.5)
        P1, E1 = _evolve(prm, P, E, 12, dt=0.25 / n, model=model, fel=0.5)
        it = _interior(prm)
        out.append((P1[it], E1[it], E[it]))
    (Pa, Ea, E0), (Pb, Eb, _) = out
    gam = prm["gam"]
    heat = np.max(np.abs(Ea[1] - E0[1]) / E0[1])
    assert heat > 0.05                                      # the test has teeth
    np.testing.assert_allclose(Pb[:2], lam * Pa[:2], rtol=1e-12)
    np.testing.assert_allclose(Eb[0], lam ** (1.0 - gam) * Ea[0], rtol=1e-12)
    np.testing.assert_allclose(Eb[1], lam ** (1.0 - el.GAM_E) * Ea[1], rtol=1e-12)


def test_proportional_partition_is_kept_on_the_torus():
    # with gamma = gamma_e, electrons holding the fraction c of the entropy and
    # receiving the fraction c of the heat keep K_e = c K_tot, through shocks,
    # floors, fixups and the E4 ceiling
    prm, P = problems.fm_torus(n1=32, n2=16, n3=4, gam=4.0 / 3.0)
    te_ti = 0.5
    c = te_ti / (1.0 + te_ti)
    E = problems.electron_scalars(P, prm["gam"], te_ti=te_ti)
    P1, E1 = _evolve(prm, P, E, 3, model=el.MODEL_CONSTANT, fel=c)
    it = _interior(prm)
    np.testing.assert_allclose(E1[1][it[1:]], c * E1[0][it[1:]], rtol=1e-12)
    assert np.all(np.isfinite(E1[it]))


@pytest.mark.parametrize("model", [el.MODEL_KAWAZURA, el.MODEL_WERNER, el.MODEL_ROWAN, el.MODEL_HOWES,
                                   el.MODEL_SHARMA])
def test_bounds_on_the_torus(model):
    prm, P = problems.fm_torus(n1=32, n2=16, n3=4)
    gam = prm["gam"]
    E = problems.electron_scalars(P, gam)
    P1, E1 = _evolve(prm, P, E, 2, model=model)
    it = _interior(prm)
    rho, u = P1[0][it[1:]], P1[1][it[1:]]
    ktot, kel = E1[0][it[1:]], E1[1][it[1:]]
    assert np.all(np.isfinite(kel))
    assert np.all(u <= el.KAPPA_MAX * rho ** gam / (gam - 1.0) * (1 + 1e-14))     # E4
    np.testing.assert_allclose(ktot, (gam - 1.0) * u / rho ** gam, rtol=1e-14)  # E5: K_tot <- K
    assert np.all(kel >= 0.0)
    assert np.all(kel <= rho ** (gam - el.GAM_E) * ktot * (1 + 1e-14))          # P_e <= P_gas


def _fe(model, beta=None, sigma=None, te_ti=1.0, gam=5.0 / 3.0, u=1.0):
    """f_e at one zone with rho = 1, internal energy u and the given beta_i (or
    sigma), T_e/T_i."""
    rho = np.array([1.0])
    u = np.array([u])
    pg = (gam - 1.0) * u
    pe = pg * te_ti / (1.0 + te_ti)
    pi = pg - pe
    bsq = 2.0 * pi / beta if beta is not None else sigma * rho
    kel = pe / rho ** el.GAM_E
    return float(el.heating_fraction(model, 0.5, rho, u, kel, bsq, gam)[0])


def test_heating_model_limits():
    # Kawazura et al. 2019: Q_i/Q_e -> 35 at high beta_i, -> 0 at low beta_i
    assert _fe(el.MODEL_KAWAZURA, beta=1e8) == pytest.approx(1.0 / 36.0, rel=1e-6)
    assert _fe(el.MODEL_KAWAZURA, beta=1e-6) == pytest.approx(1.0, abs=1e-6)
    # Werner et al. 2018: 1/4 at sigma -> 0, 1/2 at sigma -> infinity
    assert _fe(el.MODEL_WERNER, sigma=1e-12) == pytest.approx(0.25, abs=1e-6)
    assert _fe(el.MODEL_WERNER, sigma=1e12) == pytest.approx(0.5, abs=1e-6)
    # Rowan et al. 2017: 1/2 once beta_i reaches beta_max = 1/(4 sigma_w), less
    # below it (beta_i / beta_max = 8 P_i / w here: cold gas is far below)
    assert _fe(el.MODEL_ROWAN, beta=1e3) == 0.5
    assert 0.0 < _fe(el.MODEL_ROWAN, beta=1e-3, u=0.01) < 0.45
    # Howes 2010: electrons take everything at low beta_i; at high beta_i and
    # T_i = T_e, Q_i/Q_e -> 0.92 sqrt(m_p / m_e)
    assert _fe(el.MODEL_HOWES, beta=1e-3) == pytest.approx(1.0, abs=1e-12)
    assert _fe(el.MODEL_HOWES, beta=1e6) == pytest.approx(1.0 / (1.0 + 0.92 * np.sqrt(el.MP_ME)), rel=1e-6)
    # Sharma et al. 2007: Q_e/Q_i = sqrt(T_e/T_i)/3, so 1/4 at T_e = T_i and
    # 1/7 at T_i = 4 T_e; the electron share grows with T_e/T_i
    assert _fe(el.MODEL_SHARMA, beta=1.0) == pytest.approx(0.25, rel=1e-12)
    assert _fe(el.MODEL_SHARMA, beta=1.0, te_ti=0.25) == pytest.approx(1.0 / 7.0, rel=1e-12)
    assert _fe(el.MODEL_SHARMA, beta=1.0, te_ti=4.0) == pytest.approx(0.4, rel=1e-12)
    # Howes 2010 at beta_i = 1 (beta_i^x = 1 for any x): which branch of the
    # fit applies on each side of T_i = T_e (c2 = 1.2/theta, c3 = 18 for
    # T_i <= T_e; 1.6/theta and 18 + 5 log10 theta above). This checks the
    # branch selection of the reading only: the coefficients are parity unpinned.
    for r, c2, c3 in ((2.0, 1.2 * 2.0, 18.0), (0.5, 1.6 * 0.5, 18.0 + 5.0 * np.log10(2.0))):
        theta = 1.0 / r
        q = 0.92 * (c2 ** 2 + 1.0) / (c3 ** 2 + 1.0) * np.sqrt(el.MP_ME * theta) * np.exp(-1.0)
        assert _fe(el.MODEL_HOWES, beta=1.0, te_ti=r) == pytest.approx(1.0 / (1.0 + q), rel=1e-9)
    # all models are fractions
    for m in (el.MODEL_KAWAZURA, el.MODEL_WERNER, el.MODEL_ROWAN, el.MODEL_HOWES, el.MODEL_SHARMA):
        for b in (1e-8, 1e-2, 1.0, 1e2, 1e8):
            for r in (0.01, 1.0, 100.0):
                f = _fe(m, beta=b, te_ti=r)
                assert 0.0 <= f <= 1.0, (m, b, r, f)


def test_window_step_equals_the_full_step():
    # the x3-window electron step used for sampled full-size parity returns
    # the full-domain step's values on its slabs (one at the periodic seam)
    prm, P = problems.fm_torus(n1=24, n2=12, n3=20)
    E = problems.electron_scalars(P, prm["gam"], te_ti=0.5)
    g = oracle.Grid(prm)
    dt = oracle.get_dt(P, g)
    Pf, Ef, _ = el.step(P, E, g, dt, el.MODEL_KAWAZURA, 0.0)
    it = _interior(prm)
    for k0, k1 in ((0, 1), (7, 9), (19, 20)):
        Pw, Ew = el.step_window(P, E, g, dt, k0, k1, el.MODEL_KAWAZURA, 0.0)
        assert np.array_equal(Pw, Pf[it][:, k0:k1]), k0
        assert np.array_equal(Ew, Ef[it][:, k0:k1]), k0
