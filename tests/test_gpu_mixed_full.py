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
