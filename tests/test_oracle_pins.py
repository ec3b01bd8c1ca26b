"""Closed-form pins of the div B monitor and of the linear-mode frequencies.

* div B (Implementation Notes: Flux-CT keeps the corner-centred divergence of
  sqrt(-g) B at round-off): on fields built from sines the discrete corner
  divergence is an exact trigonometric expression (``problems.fields``), so
  the monitor's 1/(4 dx_d) normalisation, its transverse averaging, the sign
  of each direction's term and the sqrt(-g) weight are all fixed.
* Linear modes (Tests section: the 3D linear-mode convergence problem): the
  frequencies of a uniform magnetised state at rest follow from the
  relativistic MHD dispersion relation. With v_A^2 = b^2/(b^2 + w), c_s^2 =
  gamma p / w and mu = cos(angle between k and B):
    Alfven:     omega^2 = k^2 v_A^2 mu^2,
    fast/slow:  X^2 - [v_A^2 + c_s^2 (1 - v_A^2) + c_s^2 v_A^2 mu^2] X + c_s^2 v_A^2 mu^2 = 0,
                X = omega^2/k^2 (roots v_A^2 and c_s^2 along the field, and the
                perpendicular magnetosonic speed squared across it).
"""

import math

import numpy as np
import pytest

import oracle
import problems
from problems.fields import sine_box, sine_kerr
from problems.modes import BACKGROUND, GAMMA, load_modes, kkey
from oracle.modes import eigenmodes


# ---------------------------------------------------------------- div B

@pytest.mark.parametrize("terms", [
    ((1, 1, 1.0, 0),),                        # x1 alone: max = 2 sin(pi/16) * 16
    ((1, 1, 1.0, 2),),                        # x1, averaged over x2: * cos(pi/8)
    ((2, 1, 1.0, 0),),
    ((3, 1, 1.0, 1),),
    # a fundamental plus its first harmonic in every direction: the corner
    # divergence peaks only where all cosines are 1, so flipping the sign of
    # one direction's term (or swapping two directions' widths) lowers the max
    ((1, 1, 1.0, 0), (1, 2, 0.5, 0), (2, 1, 0.7, 0), (2, 2, 0.35, 0), (3, 1, 0.4, 0), (3, 2, 0.2, 0)),
    ((1, 1, 1.0, 3), (2, 1, 0.7, 1), (2, 2, 0.35, 0), (3, 1, 0.4, 2)),
], ids=["x1", "x1_avg_x2", "x2", "x3_avg_x1", "harmonics", "harmonics_avg"])
def test_divb_matches_closed_form_on_sines(terms):
    prm, P, div = sine_box(16, 8, 4, terms)
    g = oracle.Grid(prm)
    want = float(np.abs(div).max())
    got = oracle.divb(P, g)
    assert abs(got / want - 1.0) < 1e-13, (got, want)


def test_divb_single_direction_values():
    """The closed form itself, for the plainest case: B^1 = sin(2 pi x1) on 16
    zones has max corner divergence 2 sin(pi dx)/dx."""
    prm, P, _ = sine_box(16, 8, 4, ((1, 1, 1.0, 0),))
    assert abs(oracle.divb(P, oracle.Grid(prm)) - 2.0 * math.sin(math.pi / 16) * 16) < 1e-13


def test_divb_weights_by_sqrt_minus_g_on_kerr():
    """sqrt(-g) B^1 = sin(2 pi (x1 - x1min)/L) on a Kerr grid: the monitor sees
    the sine (the sqrt(-g) weight cancels the 1/sqrt(-g) of B^1); corners on the
    radial and polar edges are excluded."""
    prm, P, div = sine_kerr()
    g = oracle.Grid(prm)
    want = float(np.abs(div).max())
    got = oracle.divb(P, g)
    assert abs(got / want - 1.0) < 1e-13, (got, want)


def test_divb_is_zero_for_a_curl():
    """A discrete curl of a corner potential has zero corner divergence: the
    torus's initial field."""
    prm, P = problems.fm_torus(n1=32, n2=24, n3=2)
    assert oracle.divb(P, oracle.Grid(prm)) < 1e-12


# ---------------------------------------------------------------- mode frequencies

def _closed_form_omegas(kvec):
    rho, u = BACKGROUND[0], BACKGROUND[1]
    B = BACKGROUND[5:8]
    p = (GAMMA - 1.0) * u
    w = rho + u + p
    bsq = float(B @ B)                       # at rest in flat space b = (0, B)
    va2 = bsq / (bsq + w)
    cs2 = GAMMA * p / w
    k = 2.0 * math.pi * np.asarray(kvec, dtype=float)
    kk = float(np.sqrt(k @ k))
    mu2 = float((k @ B) ** 2 / (k @ k) / bsq)
    bcoef = va2 + cs2 * (1.0 - va2) + cs2 * va2 * mu2
    disc = math.sqrt(bcoef * bcoef - 4.0 * cs2 * va2 * mu2)
    xf, xs = 0.5 * (bcoef + disc), 0.5 * (bcoef - disc)
    return dict(slow=kk * math.sqrt(xs), alfven=kk * math.sqrt(va2 * mu2), fast=kk * math.sqrt(xf))


# frequencies printed for these two wave vectors (rounded to 12 decimals)
PRINTED = {
    (1, 1, 1): dict(slow=2.358963791134, alfven=3.441442325727, fast=6.929151628820),
    (1, 1, 0): dict(slow=2.410241853389, alfven=3.441442325727, fast=5.537262173313),
}


@pytest.mark.parametrize("kvec", [(1, 1, 1), (1, 1, 0)])
def test_eigenmode_frequencies_match_the_dispersion_relation(kvec):
    closed = _closed_form_omegas(kvec)
    modes = eigenmodes(BACKGROUND, GAMMA, kvec)
    table = load_modes()[kkey(kvec)]
    for name in ("slow", "alfven", "fast"):
        assert abs(closed[name] - PRINTED[kvec][name]) < 1e-11, (name, closed[name])
        assert abs(modes[name][0] / closed[name] - 1.0) < 1e-10, (name, modes[name][0], closed[name])
        assert abs(table[name]["omega"] / closed[name] - 1.0) < 1e-10, name


@pytest.mark.parametrize("kvec", [(1, 1, 1), (1, 1, 0)])
def test_eigenvectors_solve_the_linearised_problem(kvec):
    """R is a right eigenvector of the flux Jacobians: (sum_d k_d A_d) R = omega M R,
    and the Alfven mode carries no density or pressure perturbation."""
    from oracle.modes import jacobians
    M, A = jacobians(BACKGROUND, GAMMA)
    k = 2.0 * math.pi * np.asarray(kvec, dtype=float)
    K = np.einsum("d,dij->ij", k, A)
    for name, (om, R) in eigenmodes(BACKGROUND, GAMMA, kvec).items():
        res = K @ R - om * (M @ R)
        assert np.abs(res).max() < 1e-10, (name, np.abs(res).max())
    R = eigenmodes(BACKGROUND, GAMMA, kvec)["alfven"][1]
    assert abs(R[0]) < 1e-12 and abs(R[1]) < 1e-12
