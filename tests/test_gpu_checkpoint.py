"""Restart invariance on the device: stopping, writing a checkpoint, and
continuing in a fresh context gives bit for bit the run that never stopped
(for one context and for a batch), and restarting from a checkpoint of the
initial data equals starting from the initial data."""

import numpy as np
import pytest

import problems
from paper_2110_10191_amd import checkpoint

pytestmark = pytest.mark.gpu


def test_restart_equals_the_uninterrupted_run(lib, tmp_path):
    prm, P0 = problems.fm_torus(n1=48, n2=28, n3=4)
    a = lib.Sim(prm)
    Pa = a.to_device(P0)
    dt0 = a.get_dt(Pa)
    dt_a = a.run(Pa, 6, dt0)
    ref = a.to_host(Pa)
    a.close()

    b = lib.Sim(prm)
    Pb = b.to_device(P0)
    dt_b = b.run(Pb, 3, dt0)
    path = str(tmp_path / "mid.npz")
    checkpoint.save(path, prm, b.to_host(Pb), dt_b, step=3)
    b.close()

    ck = checkpoint.load(path)
    c = lib.Sim(ck.prm)
    Pc = c.to_device(ck.P)
    dt_c = c.run(Pc, 3, ck.dt)
    assert dt_c == dt_a
    assert np.array_equal(c.to_host(Pc), ref)
    c.close()


def test_checkpoint_of_the_initial_data_equals_a_fresh_start(lib, tmp_path):
    prm, P0 = problems.bondi(n1=40, n2=24, n3=2, a=0.7)
    path = str(tmp_path / "init.npz")
    s = lib.Sim(prm)
    P = s.to_device(P0)
    dt0 = s.get_dt(P)
    checkpoint.save(path, prm, s.to_host(P), dt0)
    dt_ref = s.run(P, 4, dt0)
    ref = s.to_host(P)
    s.close()
    ck = checkpoint.load(path)
    s2 = lib.Sim(ck.prm)
    P2 = s2.to_device(ck.P)
    assert s2.run(P2, 4, ck.dt) == dt_ref
    assert np.array_equal(s2.to_host(P2), ref)
    s2.close()


def test_batch_restart(lib, tmp_path):
    jobs = [problems.fm_torus(n1=48, n2=28, n3=4), problems.linear_modes(n=12, n3=9, kvec=(1, 1, 0))]

    def start():
        sims = [lib.Sim(prm) for prm, _ in jobs]
        states = [s.to_device(P0) for s, (_, P0) in zip(sims, jobs)]
        return sims, states

    sims, states = start()
    dt0 = [s.get_dt(P) for s, P in zip(sims, states)]
    b = lib.Batch(sims)
    b.set_dt(dt0)
    b.step(states, nsteps=4)
    dts_ref, _ = b.get()
    refs = [s.to_host(P) for s, P in zip(sims, states)]
    b.close()

    sims, states = start()
    b = lib.Batch(sims)
    b.set_dt(dt0)
    b.step(states, nsteps=2)
    dts, _ = b.get()
    paths = []
    for j, (s, P) in enumerate(zip(sims, states)):
        paths.append(str(tmp_path / f"job{j}.npz"))
        checkpoint.save(paths[-1], s.prm, s.to_host(P), dts[j], step=2)
    b.close()
    for s in sims:
        s.close()

    cks = [checkpoint.load(p) for p in paths]
    sims = [lib.Sim(ck.prm) for ck in cks]
    states = [s.to_device(ck.P) for s, ck in zip(sims, cks)]
    b = lib.Batch(sims)
    b.set_dt([ck.dt for ck in cks])
    b.step(states, nsteps=2)
    dts2, _ = b.get()
    assert dts2 == dts_ref
    for s, P, ref in zip(sims, states, refs):
        assert np.array_equal(s.to_host(P), ref)
    b.close()


def test_restart_with_electron_heating(lib, tmp_path):
    """A run with electron heating stopped, written (primitives, entropies,
    model) and continued in a fresh context equals the run that never stopped."""
    prm, P0 = problems.fm_torus(n1=48, n2=28, n3=4)
    E0 = problems.electron_scalars(P0, prm["gam"], te_ti=0.5)
    heat = ("howes", 0.0)
    a = lib.Sim(prm)
    Pa, Ea = a.to_device(P0), a.to_device(E0)
    dt0 = a.get_dt(Pa)
    dt_a = a.run_electrons(Pa, Ea, 6, dt0, *heat)
    ref_P, ref_E = a.to_host(Pa), a.to_host(Ea)
    a.close()

    b = lib.Sim(prm)
    Pb, Eb = b.to_device(P0), b.to_device(E0)
    dt_b = b.run_electrons(Pb, Eb, 3, dt0, *heat)
    path = str(tmp_path / "mid_e.npz")
    checkpoint.save(path, prm, b.to_host(Pb), dt_b, step=3, E=b.to_host(Eb), heat=heat)
    b.close()

    ck = checkpoint.load(path)
    c = lib.Sim(ck.prm)
    Pc, Ec = c.to_device(ck.P), c.to_device(ck.E)
    dt_c = c.run_electrons(Pc, Ec, 3, ck.dt, *ck.heat)
    assert dt_c == dt_a
    assert np.array_equal(c.to_host(Pc), ref_P) and np.array_equal(c.to_host(Ec), ref_E)
    c.close()
