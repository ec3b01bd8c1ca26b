"""Decomposition invariance on one device: the problem split along x3 into
parts that exchange three ghost planes per substep (the multi-device layout)
evolves bit for bit like the single context, step sizes included."""

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
    if fails:
        pytest.skip(f"{fails} failed inversions: the fixup near a part boundary differs by design")
    assert np.array_equal(got, want)
    split.close()
    ref.close()


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
