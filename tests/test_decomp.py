"""Host-side checks of the x3 split (no device needed: the problem is
rejected before any context is made)."""

import pytest

import problems
from paper_2110_10191_amd.decomp import SlabSplit


@pytest.mark.parametrize("edit,needle", [
    (dict(n3=9), "multiple"),
    (dict(bc=[[0, 0], [0, 0], [3, 3]]), "periodic x3"),
    (dict(n3=4), "at least"),
])
def test_split_rejects(edit, needle):
    prm, P0 = problems.linear_modes(n=8)
    prm = dict(prm, **edit)
    with pytest.raises(ValueError, match=needle):
        SlabSplit(prm, P0, 2 if edit.get("n3") != 4 else 4)


def test_split_rejects_geometry_that_depends_on_x3():
    # Cartesian Kerr-Schild tables are 3D: a part's tables, built from its own
    # x3 extent, would match the whole domain's only to rounding
    prm, P0 = problems.cks_bondi(8, 8, 8)
    prm = dict(prm, bc=[[3, 3], [3, 3], [0, 0]])
    with pytest.raises(ValueError, match="does not depend on x3"):
        SlabSplit(prm, P0, 2)
