"""Block tiles are a launch parameter only: every zone and face is computed by
one thread from the same operands, and the only cross-thread reductions are
maxima and counts, so any legal tile gives bitwise the same evolution."""

import numpy as np
import pytest

import problems

pytestmark = pytest.mark.gpu

SWEEP_TILES = [(64, 8), (32, 2), (16, 4), (128, 2), (256, 1), (64, 1), (128, 4), (32, 16)]
UPDATE_TILES = [(64, 4), (32, 8), (128, 1), (64, 1), (256, 1), (128, 2), (16, 4), (32, 2)]


def evolve(lib, prm, P0, nsteps, sweep=None, update=None):
    sim = lib.Sim(prm)
    if sweep:
        sim.set_tiles("sweep", *sweep)
    if update:
        sim.set_tiles("update", *update)
    P = sim.to_device(P0)
    dt = sim.get_dt(P)
    for _ in range(nsteps):
        dt = min(sim.step(P, dt), 1.3 * dt)
    out = sim.to_host(P)
    sim.close()
    return out, dt


@pytest.mark.parametrize("make", [
    lambda: problems.fm_torus(n1=72, n2=20, n3=5),
    lambda: problems.fm_torus(n1=40, n2=18, n3=3, recon=problems.RECON_WENO5, precision=problems.MIXED),
    # FP64 WENO5 stages the widest LDS tiles: 128 x 4 and 256 x 1 need more
    # than the default 64 KiB a block (76.6 and 100 KB)
    lambda: problems.fm_torus(n1=40, n2=18, n3=3, recon=problems.RECON_WENO5),
    lambda: problems.bondi(n1=37, n2=13, n3=2, a=0.5),
], ids=["torus_mc_fp64", "torus_weno5_mixed", "torus_weno5_fp64", "bondi"])
def test_any_tile_gives_the_same_bits(lib, make):
    prm, P0 = make()
    ref, dt_ref = evolve(lib, prm, P0, 3)
    for st, ut in zip(SWEEP_TILES[1:], UPDATE_TILES[1:]):
        out, dt = evolve(lib, prm, P0, 3, sweep=st, update=ut)
        assert dt == dt_ref, (st, ut)
        assert np.array_equal(out, ref), (st, ut)


def test_tile_validation(lib):
    prm, _ = problems.linear_modes(n=8)
    sim = lib.Sim(prm)
    assert sim.get_tiles("sweep") == (64, 8)
    assert sim.get_tiles("update") == (64, 1)
    for bad in [(48, 4), (32, 3), (512, 1), (8, 8), (16, 3), (0, 4), (64, 0), (64, 16)]:
        with pytest.raises(lib.GrmhdError):
            sim.set_tiles("sweep", *bad)
    for bad in [(64, 8), (128, 4), (32, 16)]:                  # above the update's 256 threads
        with pytest.raises(lib.GrmhdError):
            sim.set_tiles("update", *bad)
    with pytest.raises(lib.GrmhdError):
        sim.set_tiles(7, 64, 4)
    sim.set_tiles("update", 128, 2)
    sim.set_tiles("sweep", 128, 4)
    assert sim.get_tiles("update") == (128, 2)
    assert sim.get_tiles("sweep") == (128, 4)
    sim.close()


def test_batch_uses_its_first_jobs_tiles(lib):
    jobs = [problems.fm_torus(n1=48, n2=28, n3=4), problems.linear_modes(n=12, n3=9, kvec=(1, 1, 0))]
    refs = [evolve(lib, prm, P0, 2)[0] for prm, P0 in jobs]
    sims = [lib.Sim(prm) for prm, _ in jobs]
    sims[0].set_tiles("sweep", 128, 4)
    sims[0].set_tiles("update", 32, 2)
    states = [s.to_device(P0) for s, (_, P0) in zip(sims, jobs)]
    dt0 = [s.get_dt(P) for s, P in zip(sims, states)]
    b = lib.Batch(sims)
    b.set_dt(dt0)
    b.step(states, nsteps=2)
    _, status = b.get()
    assert status == [0, 0]
    for s, P, ref in zip(sims, states, refs):
        assert np.array_equal(s.to_host(P), ref)
    b.close()
    for s in sims:
        s.close()
