"""Decomposition invariance on one device (Tests section: evolution identical
across decompositions): the problem split along x3 into parts that exchange
three ghost planes per substep, and the new boundary planes with their failure
flags before the fixup (the multi-device layout), evolves bit for bit like the
single context, step sizes included, also where inversions fail next to part
boundaries; checkpoints move between decompositions."""

import numpy as np
import pytest

import problems
from paper_2110_10191_amd.decomp import SlabSplit

pytestmark = pytest.mark.gpu
NG = 3


def interior(P, prm):
    return P[:, NG:NG + prm["n3"], NG:NG + prm["n2"], NG:NG + prm["n1"]]


@pytest.mark.parametrize("make,parts", [
    (lambda: problems.linear_modes(n=32), 2),
    (lambda: problems.linear_modes(n=32), 4),
    (lambda: problems.fm_torus(n1=48, n2=28, n3=8), 2),
    (lambda: problems.fm_torus(n1=40, n2=18, n3=8, recon=problems.RECON_WENO5, precision=problems.MIXED), 2),
], ids=["box_2", "box_4", "torus_2", "torus_weno5_mixed_2"])
def test_split_equals_single_context(lib, make, parts):
    prm, P0 = make()
    ref = lib.Sim(prm)
    P = ref.to_device(P0)
    dt = ref.get_dt(P)
    split = SlabSplit(prm, P0, parts)
    fails = 0
    for _ in range(4):
        dt_ref = min(ref.step(P, dt), 1.3 * dt)
        fails += ref.step_failures()
        dt_split = min(split.step(dt), 1.3 * dt)
        assert dt_split == dt_ref
        dt = dt_ref
    got = split.to_host()
    want = interior(ref.to_host(P), prm)
    print("failed inversions", fails)
    assert np.array_equal(got, want)
    split.close()
    ref.close()


def run_single(lib, prm, P0, dt, nsteps):
    sim = lib.Sim(prm)
    P = sim.to_device(P0)
    fails = 0
    for _ in range(nsteps):
        dt = min(sim.step(P, dt), 1.3 * dt)
        fails += sim.step_failures()
    out = interior(sim.to_host(P), prm)
    sim.close()
    return out, dt, fails


def run_split(prm, P0, parts, dt, nsteps):
    split = SlabSplit(prm, P0, parts)
    for _ in range(nsteps):
        dt = min(split.step(dt), 1.3 * dt)
    out = split.to_host()
    split.close()
    return out, dt


@pytest.mark.parametrize("make,parts,planes", [
    (lambda: problems.linear_modes(n=32), 2, (15, 16, 0, 31)),
    (lambda: problems.linear_modes(n=32), 4, (7, 8, 24)),
    (lambda: problems.fm_torus(n1=48, n2=28, n3=8), 2, (3, 4, 0)),
    (lambda: problems.fm_torus(n1=40, n2=18, n3=16, recon=problems.RECON_WENO5, precision=problems.MIXED), 4,
     (3, 4, 12, 15)),
], ids=["box_2", "box_4", "torus_2", "torus_weno5_mixed_4"])
def test_split_with_failures_at_part_boundaries(lib, make, parts, planes):
    """Zones whose inversion fails on both sides of the part boundaries and at
    the periodic seam (a NaN internal energy in each listed x3 plane makes a
    cross of zones around it fail; the fixup repairs them): the split run still
    equals the single context bit for bit, because the fixup sees the same 26
    neighbours across part boundaries and across the seam."""
    prm, P0 = make()
    P0 = P0.copy()
    for m, k in enumerate(planes):
        P0[1, NG + k, NG + 3 + 2 * m, NG + 5 + 3 * m] = np.nan
    sim = lib.Sim(prm)
    dt = sim.get_dt(sim.to_device(make()[1]))           # the step size of the clean state
    sim.close()
    want, dt_want, fails = run_single(lib, prm, P0, dt, 3)
    got, dt_got = run_split(prm, P0, parts, dt, 3)
    print("failed inversions", fails, "dt", dt_want)
    assert fails > 0
    assert np.isfinite(want).all()
    assert dt_got == dt_want
    assert np.array_equal(got, want)


def test_checkpoint_moves_between_decompositions(lib, tmp_path):
    """A checkpoint written by a run split in 2 parts restarts in 4 parts and in
    one context; all three continuations equal the run that never stopped,
    bit for bit (with failed zones at part boundaries along the way)."""
    from paper_2110_10191_amd import checkpoint
    prm, P0 = problems.fm_torus(n1=48, n2=28, n3=16)
    sim = lib.Sim(prm)
    dt0 = sim.get_dt(sim.to_device(P0))                    # the step size of the clean state
    sim.close()
    P0 = P0.copy()
    P0[1, NG + 7, NG + 6, NG + 9] = np.nan                # fails next to the 2-part boundary
    P0[1, NG + 4, NG + 8, NG + 12] = np.nan               # and next to a 4-part boundary
    want, dt_want, fails = run_single(lib, prm, P0, dt0, 6)
    assert fails > 0
    half, dt_half = run_split(prm, P0, 2, dt0, 3)
    Pck = np.zeros_like(P0)
    Pck[:, NG:NG + 16, NG:NG + 28, NG:NG + 48] = half
    path = str(tmp_path / "split2.npz")
    checkpoint.save(path, prm, Pck, dt_half, step=3)
    ck = checkpoint.load(path)
    four, dt_four = run_split(ck.prm, ck.P, 4, ck.dt, 3)
    one, dt_one, _ = run_single(lib, ck.prm, ck.P, ck.dt, 3)
    assert dt_four == dt_want and dt_one == dt_want
    assert np.array_equal(four, want)
    assert np.array_equal(one, want)


def test_split_rejects_what_it_cannot_reproduce(lib):
    prm, P0 = problems.linear_modes(n=32)
    with pytest.raises(ValueError):
        SlabSplit(prm, P0, 3)                  # 32 planes do not split in 3
    with pytest.raises(ValueError):
        SlabSplit(prm, P0, 16)                 # 2 planes a part, fewer than the ghost depth
    prm_b, P0_b = problems.bondi(n1=40, n2=24, n3=4)
    prm_b = dict(prm_b, bc=[prm_b["bc"][0], prm_b["bc"][1], [3, 3]])
    with pytest.raises(ValueError):
        SlabSplit(prm_b, P0_b, 2)              # x3 not periodic
