"""The benchmark configuration at full size against the oracle.

288 x 128 x 128 FMKS torus (a = 0.9375, beta = 100, seeded 4 % noise on u),
10 steps:

* FP64 with MC reconstruction through grmhd_run, the call and launch
  configuration the benchmark times, from the oracle's first Courant step
  (the device then keeps its own step sizes, which agree with the oracle's to
  rounding): relative L1 <= 1e-10 per primitive;
* mixed precision (FP32 reconstruction, fluxes and EMFs) with WENO5, stepped
  with the FP64 WENO5 oracle's step sizes: relative L1 <= 1e-5 per primitive,
  with the largest local error printed.

The oracle runs by x3 slabs in worker processes (``oracle.slabs``), which
reproduces its whole-domain step bit for bit. The velocity components are
also compared with an error normalised by the L1 norm of all three, which
stays well posed for a component that is physically near zero (u~2 in the
equatorial torus).
"""

import numpy as np
import pytest

import problems
from oracle import slabs

NG = 3
NSTEPS = 10
pytestmark = pytest.mark.gpu


def interior(P, prm):
    return P[:, NG:NG + prm["n3"], NG:NG + prm["n2"], NG:NG + prm["n1"]]


def rel_l1(a, b):
    out = []
    for v in range(a.shape[0]):
        num = np.abs(a[v] - b[v]).sum()
        den = np.abs(b[v]).sum()
        out.append(num / den if den > 0 else (0.0 if num == 0 else np.inf))
    return np.array(out)


def velocity_l1(a, b):
    """sum |du~^i| / sum_j sum |u~^j| for i = 1..3."""
    den = sum(np.abs(b[2 + j]).sum() for j in range(3))
    return np.array([np.abs(a[2 + i] - b[2 + i]).sum() / den for i in range(3)])


def max_local(a, b):
    """max |a - b| over max |b|, per primitive."""
    return np.array([np.abs(a[v] - b[v]).max() / max(np.abs(b[v]).max(), 1e-300) for v in range(a.shape[0])])


def log(msg):
    print(msg, flush=True)


def test_full_size_torus_ten_steps_fp64_mc_run(lib):
    prm, P0 = problems.fm_torus()
    ref, dts, fails = slabs.run(prm, P0, NSTEPS, log=log)
    sim = lib.Sim(prm)
    P = sim.to_device(P0)
    dt_next = sim.run(P, NSTEPS, dts[0])
    got = interior(sim.to_host(P), prm)
    sim.close()
    want = interior(ref, prm)
    err = rel_l1(got, want)
    verr = velocity_l1(got, want)
    print("oracle step sizes", dts, "failed inversions", fails)
    print("rel-L1", err)
    print("velocity error / L1 of all three components", verr)
    print("max local", max_local(got, want))
    print("device dt after 10 steps", dt_next)
    assert np.isfinite(got).all()
    assert (err <= 1e-10).all(), err
    assert (verr <= 1e-10).all(), verr


def test_full_size_torus_ten_steps_mixed_weno5(lib):
    prm64, P0 = problems.fm_torus(recon=problems.RECON_WENO5)
    ref, dts, fails = slabs.run(prm64, P0, NSTEPS, log=log)
    prm = dict(prm64, precision=problems.MIXED)
    sim = lib.Sim(prm)
    P = sim.to_device(P0)
    for dt in dts:
        sim.step(P, dt, want_dt_next=False)
    got = interior(sim.to_host(P), prm)
    sim.close()
    want = interior(ref, prm64)
    err = rel_l1(got, want)
    print("oracle step sizes", dts, "failed inversions", fails)
    print("mixed WENO5 rel-L1 vs FP64 oracle", err)
    print("velocity error / L1 of all three components", velocity_l1(got, want))
    print("max local (max |diff| / max |value|)", max_local(got, want))
    assert np.isfinite(got).all()
    assert (err <= 1e-5).all(), err
