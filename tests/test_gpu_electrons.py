"""Parity of the electron-heating step (grmhd_step_electrons, through the C
ABI) with the oracle's electron step.

Bar as for the fluid step: relative L1 per variable <= 1e-10 after the steps
(FP64), <= 1e-5 in mixed precision, both sides driven by the oracle's
time-step sequence. Sizes span several tiles with ragged tails."""

import numpy as np
import pytest

import oracle
import problems
from oracle import electrons as el

NG = 3
pytestmark = pytest.mark.gpu


def interior(A, prm):
    return A[:, NG:NG + prm["n3"], NG:NG + prm["n2"], NG:NG + prm["n1"]]


def rel_l1(a, b):
    out = []
    for v in range(a.shape[0]):
        num = np.abs(a[v] - b[v]).sum()
        den = np.abs(b[v]).sum()
        out.append(num / den if den > 0 else (0.0 if num == 0 else np.inf))
    return np.array(out)


def oracle_run(prm, P0, E0, nsteps, model, fel):
    g = oracle.Grid(prm)
    dt = oracle.get_dt(P0, g)
    P, E, dts = P0, E0, []
    for _ in range(nsteps):
        dts.append(dt)
        P, E, dn = el.step(P, E, g, dt, model, fel)
        dt = min(dn, 1.3 * dt)
    return P, E, dts, dn


def gpu_run(lib, prm, P0, E0, dts, model, fel):
    sim = lib.Sim(prm)
    P, E = sim.to_device(P0), sim.to_device(E0)
    dn = None
    for dt in dts:
        dn = sim.step_electrons(P, E, dt, model, fel)
    out = sim.to_host(P), sim.to_host(E)
    sim.close()
    return out[0], out[1], dn


CASES = {
    "torus_mc_const": (lambda: problems.fm_torus(n1=72, n2=20, n3=5), el.MODEL_CONSTANT, 0.3, 6),
    "torus_mc_kawazura": (lambda: problems.fm_torus(n1=72, n2=20, n3=5), el.MODEL_KAWAZURA, 0.0, 6),
    "torus_mc_werner": (lambda: problems.fm_torus(n1=40, n2=18, n3=3), el.MODEL_WERNER, 0.0, 6),
    "torus_mc_rowan": (lambda: problems.fm_torus(n1=40, n2=18, n3=3), el.MODEL_ROWAN, 0.0, 6),
    "torus_mc_howes": (lambda: problems.fm_torus(n1=72, n2=20, n3=5), el.MODEL_HOWES, 0.0, 6),
    "torus_mc_sharma": (lambda: problems.fm_torus(n1=40, n2=18, n3=3), el.MODEL_SHARMA, 0.0, 6),
    "torus_weno5_howes": (lambda: problems.fm_torus(n1=72, n2=20, n3=5, recon=problems.RECON_WENO5),
                          el.MODEL_HOWES, 0.0, 6),
    "bondi_kawazura": (lambda: problems.bondi(n1=37, n2=13, n3=2, a=0.5), el.MODEL_KAWAZURA, 0.0, 10),
    "box_const": (lambda: problems.linear_modes(n=24, n3=6, amp=1e-3), el.MODEL_CONSTANT, 0.5, 10),
}


@pytest.mark.parametrize("case", list(CASES))
def test_electron_step_matches_oracle(lib, case):
    make, model, fel, nsteps = CASES[case]
    prm, P0 = make()
    E0 = problems.electron_scalars(P0, prm["gam"], te_ti=0.5)
    Pr, Er, dts, dn_r = oracle_run(prm, P0, E0, nsteps, model, fel)
    Pg, Eg, dn_g = gpu_run(lib, prm, P0, E0, dts, model, fel)
    eP = rel_l1(interior(Pg, prm), interior(Pr, prm))
    eE = rel_l1(interior(Eg, prm), interior(Er, prm))
    print(case, "P", eP.max(), "E", eE)
    assert eP.max() <= 1e-10, eP
    assert eE.max() <= 1e-10, eE
    assert dn_g == pytest.approx(dn_r, rel=1e-10)


def test_electron_step_mixed_precision(lib):
    prm, P0 = problems.fm_torus(n1=72, n2=20, n3=5, recon=problems.RECON_WENO5, precision=problems.MIXED)
    E0 = problems.electron_scalars(P0, prm["gam"], te_ti=0.5)
    ref_prm = dict(prm, precision=problems.FP64)
    Pr, Er, dts, _ = oracle_run(ref_prm, P0, E0, 6, el.MODEL_KAWAZURA, 0.0)
    Pg, Eg, _ = gpu_run(lib, prm, P0, E0, dts, el.MODEL_KAWAZURA, 0.0)
    eP = rel_l1(interior(Pg, prm), interior(Pr, prm))
    eE = rel_l1(interior(Eg, prm), interior(Er, prm))
    print("mixed P", eP.max(), "E", eE)
    assert eP.max() <= 1e-5 and eE.max() <= 1e-5, (eP, eE)


def test_fluid_is_the_plain_step_where_the_ceiling_is_inactive(lib):
    # the electron passes only read the fluid, apart from the u ceiling, which
    # this flow never reaches: the primitives are grmhd_step's bit for bit
    prm, P0 = problems.linear_modes(n=24, n3=6, amp=1e-3)
    E0 = problems.electron_scalars(P0, prm["gam"])
    sim = lib.Sim(prm)
    Pa, E, Pb = sim.to_device(P0), sim.to_device(E0), sim.to_device(P0)
    dt = sim.get_dt(Pa)
    for _ in range(4):
        da = sim.step_electrons(Pa, E, dt, "werner")
        db = sim.step(Pb, dt)
        assert da == db
        dt = min(da, 1.3 * dt)
    assert np.array_equal(sim.to_host(Pa), sim.to_host(Pb))
    sim.close()


def test_argument_errors(lib):
    prm, P0 = problems.linear_modes(n=8)
    sim = lib.Sim(prm)
    P, E = sim.to_device(P0), sim.to_device(problems.electron_scalars(P0, prm["gam"]))
    for model, fel in [(6, 0.5), (-1, 0.5), (0, 1.5), (0, -0.1), (0, float("nan"))]:
        with pytest.raises(lib.GrmhdError) as e:
            sim.step_electrons(P, E, 1e-3, model, fel)
        assert e.value.status == lib.GRMHD_EINVAL
    with pytest.raises(lib.GrmhdError):
        lib.grmhd_step_electrons(sim.ctx, P, None, 1e-3)
    with pytest.raises(lib.GrmhdError):
        sim.step_electrons(P, E, 0.0)
    sim.step_electrons(P, E, 1e-3, "howes", 7.0)      # fel is ignored by the models
    sim.close()


def test_full_size_torus_sampled_slabs(lib):
    """The benchmark's electron configuration (288 x 128 x 128 FMKS torus, MC,
    FP64, host-driven grmhd_step_electrons, default tiles), Howes model: one
    GPU step compared on two x3 slabs (one at the periodic seam) that the
    oracle computes from windows of the same initial state."""
    prm, P0 = problems.fm_torus()
    E0 = problems.electron_scalars(P0, prm["gam"], te_ti=0.5)
    g = oracle.Grid(prm)
    dt = 0.005
    sim = lib.Sim(prm)
    P, E = sim.to_device(P0), sim.to_device(E0)
    sim.step_electrons(P, E, dt, el.MODEL_HOWES, 0.0, want_dt_next=False)
    Pg, Eg = interior(sim.to_host(P), prm), interior(sim.to_host(E), prm)
    sim.close()
    for k0 in (0, 77):
        Pr, Er = el.step_window(P0, E0, g, dt, k0, k0 + 1, el.MODEL_HOWES, 0.0)
        eP = rel_l1(Pg[:, k0:k0 + 1], Pr)
        eE = rel_l1(Eg[:, k0:k0 + 1], Er)
        print("slab", k0, eP.max(), eE)
        assert eP.max() <= 1e-10 and eE.max() <= 1e-10, (k0, eP, eE)


def test_run_electrons_equals_the_host_loop(lib):
    """grmhd_run_electrons keeps the step size on the device and gives the
    same bits as a host loop of dt <- min(dt_next, 1.3 dt) around
    grmhd_step_electrons."""
    prm, P0 = problems.fm_torus(n1=72, n2=20, n3=5)
    E0 = problems.electron_scalars(P0, prm["gam"], te_ti=0.5)
    sim = lib.Sim(prm)
    Pa, Ea = sim.to_device(P0), sim.to_device(E0)
    Pb, Eb = sim.to_device(P0), sim.to_device(E0)
    dt0 = sim.get_dt(Pa)
    dt = dt0
    for _ in range(5):
        dt = min(sim.step_electrons(Pa, Ea, dt, "howes"), 1.3 * dt)
    dt_dev = sim.run_electrons(Pb, Eb, 5, dt0, "howes")
    assert dt_dev == dt
    assert np.array_equal(sim.to_host(Pa), sim.to_host(Pb))
    assert np.array_equal(sim.to_host(Ea), sim.to_host(Eb))
    with pytest.raises(lib.GrmhdError):
        sim.run_electrons(Pb, Eb, 1, dt, 9)
    sim.close()


@pytest.mark.parametrize("make,model,fel", [
    (lambda: problems.linear_modes(n=67, n3=2, amp=1e-3), el.MODEL_SHARMA, 0.0),     # ragged tiles, thin x3
    (lambda: problems.linear_modes(n=64, n3=1, amp=1e-3), el.MODEL_CONSTANT, 1.0),   # exact tiles, one plane
    (lambda: problems.fm_torus(n1=48, n2=3, n3=2), el.MODEL_KAWAZURA, 0.0),          # smallest polar grid
    (lambda: problems.fm_torus(n1=130, n2=9, n3=3, recon=problems.RECON_WENO5), el.MODEL_ROWAN, 0.0),
], ids=["ragged", "one_plane", "polar_n2_3", "weno5_ragged"])
def test_electron_edge_shapes(lib, make, model, fel):
    prm, P0 = make()
    E0 = problems.electron_scalars(P0, prm["gam"], te_ti=0.5)
    Pr, Er, dts, _ = oracle_run(prm, P0, E0, 3, model, fel)
    Pg, Eg, _ = gpu_run(lib, prm, P0, E0, dts, model, fel)
    eP = rel_l1(interior(Pg, prm), interior(Pr, prm))
    eE = rel_l1(interior(Eg, prm), interior(Er, prm))
    print("edge", prm["n1"], prm["n2"], prm["n3"], eP.max(), eE)
    assert eP.max() <= 1e-10 and eE.max() <= 1e-10, (eP, eE)


def test_electron_step_is_deterministic_and_tile_independent(lib):
    """Two runs give the same bits, and so does every legal update tile (the
    electron passes run on the update's tiles; each zone is one thread's work)."""
    prm, P0 = problems.fm_torus(n1=72, n2=20, n3=5)
    E0 = problems.electron_scalars(P0, prm["gam"], te_ti=0.5)
    outs = []
    for tile in [(64, 4), (64, 4), (32, 8), (128, 2), (16, 4)]:
        sim = lib.Sim(prm)
        sim.set_tiles("update", *tile)
        P, E = sim.to_device(P0), sim.to_device(E0)
        dt = sim.run_electrons(P, E, 3, sim.get_dt(P), "kawazura")
        outs.append((sim.to_host(P), sim.to_host(E), dt))
        sim.close()
    for P, E, dt in outs[1:]:
        assert np.array_equal(P, outs[0][0]) and np.array_equal(E, outs[0][1]) and dt == outs[0][2]


def test_full_size_mixed_precision_slab(lib):
    """Mixed precision (FP32 faces, WENO5) with electron heating on the full
    288 x 128 x 128 torus: one step against the FP64 oracle on an x3 slab,
    within the mixed-precision bar."""
    prm, P0 = problems.fm_torus(recon=problems.RECON_WENO5, precision=problems.MIXED)
    E0 = problems.electron_scalars(P0, prm["gam"], te_ti=0.5)
    dt = 0.005
    sim = lib.Sim(prm)
    P, E = sim.to_device(P0), sim.to_device(E0)
    sim.step_electrons(P, E, dt, el.MODEL_KAWAZURA, 0.0, want_dt_next=False)
    Pg, Eg = interior(sim.to_host(P), prm), interior(sim.to_host(E), prm)
    sim.close()
    g = oracle.Grid(dict(prm, precision=problems.FP64))
    Pr, Er = el.step_window(P0, E0, g, dt, 40, 41, el.MODEL_KAWAZURA, 0.0)
    eP = rel_l1(Pg[:, 40:41], Pr)
    eE = rel_l1(Eg[:, 40:41], Er)
    print("mixed slab 40", eP.max(), eE)
    assert eP.max() <= 1e-5 and eE.max() <= 1e-5, (eP, eE)
