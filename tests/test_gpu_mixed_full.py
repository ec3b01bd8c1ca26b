"""Mixed precision on the full torus configuration (288 x 128 x 128 FMKS,
WENO5): FP32 reconstruction, face fluxes and EMFs, FP64 accumulation, metric,
source and inversion. Error statement per primitive:

* after 10 steps against the FP64 path (which matches the oracle to 1e-10 on
  every configuration the oracle can run): relative L1 <= 1e-5;
* after 1 step against the oracle itself on an x3 slab.
"""

import numpy as np
import pytest

import oracle
import problems

NG = 3
pytestmark = pytest.mark.gpu


def interior(P, prm):
    return P[:, NG:NG + prm["n3"], NG:NG + prm["n2"], NG:NG + prm["n1"]]


def rel_l1(a, b):
    num = np.abs(a - b).reshape(a.shape[0], -1).sum(1)
    den = np.abs(b).reshape(a.shape[0], -1).sum(1)
    return num / den


def evolve(lib, prm, P0, dts):
    sim = lib.Sim(prm)
    P = sim.to_device(P0)
    for dt in dts:
        sim.step(P, dt, want_dt_next=False)
    out = sim.to_host(P)
    sim.close()
    return out


def test_mixed_vs_fp64_ten_steps(lib):
    prm64, P0 = problems.fm_torus(recon=problems.RECON_WENO5)
    prm32 = dict(prm64, precision=problems.MIXED)
    dts = [0.005] * 10          # fixed steps below the grid's Courant limit (~0.01)
    ref = interior(evolve(lib, prm64, P0, dts), prm64)
    got = interior(evolve(lib, prm32, P0, dts), prm32)
    err = rel_l1(got, ref)
    maxrel = np.abs(got - ref).reshape(8, -1).max(1) / np.abs(ref).reshape(8, -1).max(1)
    print("mixed vs fp64, 10 steps: rel-L1", err, "max |diff| / max |ref|", maxrel)
    assert (err <= 1e-5).all(), err


def test_mixed_one_step_vs_oracle_slab(lib):
    prm64, P0 = problems.fm_torus(recon=problems.RECON_WENO5)
    prm32 = dict(prm64, precision=problems.MIXED)
    dt = 0.005
    got = interior(evolve(lib, prm32, P0, [dt]), prm32)
    ref = oracle.step_window(P0, oracle.Grid(prm64), dt, 40, 41)
    err = rel_l1(got[:, 40:41], ref)
    print("mixed vs oracle, 1 step, slab 40:", err)
    assert (err <= 1e-5).all(), err


def _mode_error(lib, n, precision, recon, T=0.5):
    from problems.modes import mode_solution
    prm, P0 = problems.linear_modes(n=n, kvec=(1, 1, 0), n3=1, recon=recon, precision=precision)
    sim = lib.Sim(prm)
    P = sim.to_device(P0)
    t, dt = 0.0, sim.get_dt(P)
    while t < T - 1e-14:
        dt = min(dt, T - t)
        dn = sim.step(P, dt)
        t += dt
        dt = min(dn, 1.3 * dt)
    out = interior(sim.to_host(P), prm)
    sim.close()
    return float(np.abs(out - mode_solution(prm, T)).mean())


@pytest.mark.parametrize("recon", [problems.RECON_MC, problems.RECON_WENO5], ids=["mc", "weno5"])
def test_modes_convergence_fp64_and_mixed(lib, recon):
    """Linear modes (amplitude 1e-4 on an O(1) background, k = 2 pi (1, 1, 0)):
    the FP64 path converges at second order down to n = 128; the mixed path
    follows it while the truncation error dominates and then levels off at the
    FP32 rounding floor, about 1e-7 of the background."""
    ns = (16, 32, 64, 128)
    e64 = [_mode_error(lib, n, problems.FP64, recon) for n in ns]
    e32 = [_mode_error(lib, n, problems.MIXED, recon) for n in ns]
    s64 = np.log2(np.array(e64[:-1]) / np.array(e64[1:]))
    print("fp64", e64, s64, "mixed", e32)
    assert (s64 > 1.9).all(), (e64, s64)
    assert abs(e32[0] / e64[0] - 1.0) < 0.05, (e32, e64)
    assert max(e32) < 1e-6 and e32[-1] < 1.5e-7, e32
