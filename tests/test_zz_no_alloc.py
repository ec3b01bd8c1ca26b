"""grmhd_divb_noalloc: the div B monitor with its partial maxima in the
library's static device scratch instead of context memory. Checked against
grmhd_divb on two calls in a row, the second on a smaller grid (the array
keeps the first call's slots, which the second must not see), and its size
limit."""

import numpy as np
import pytest

import problems
from problems import fields

pytestmark = pytest.mark.gpu


def test_noalloc_divb_equals_divb_on_two_calls(lib):
    big = fields.sine_box(67, 9, 5, ((1, 1, 1.0, 3), (2, 1, 0.7, 1), (2, 2, 0.35, 0), (3, 1, 0.4, 2)))
    small = fields.sine_kerr(n1=32, n2=16, n3=4)
    prm_t, P_t = problems.fm_torus(n1=72, n2=40, n3=6)
    seen = []
    for prm, P0 in ((big[0], big[1]), (small[0], small[1]), (prm_t, P_t)):
        sim = lib.Sim(prm)
        P = sim.to_device(P0)
        a = lib.grmhd_divb_noalloc(sim.ctx, P)
        b = lib.grmhd_divb(sim.ctx, P)
        print(prm["n1"], prm["n2"], prm["n3"], "noalloc", a, "divb", b)
        assert a == b
        seen.append(a)
        sim.close()
    # the second (smaller) grid's maximum is below the first's: a stale slot
    # of the first call would have shown
    assert seen[1] < seen[0]
    assert seen[2] < 1e-12


def test_noalloc_divb_full_size_torus(lib):
    """The benchmark torus (288 x 128 x 128 needs 20480 of the 65536 slots)."""
    prm, P0 = problems.fm_torus()
    sim = lib.Sim(prm)
    P = sim.to_device(P0)
    a = lib.grmhd_divb_noalloc(sim.ctx, P)
    assert a == lib.grmhd_divb(sim.ctx, P)
    assert a < 1e-12
    sim.close()


def test_noalloc_divb_rejects_a_grid_beyond_the_scratch(lib):
    """256 x 256 x 257 needs 4 * 64 * 257 = 65792 slots: EINVAL, and nothing is
    launched (the state argument is never read)."""
    import torch
    prm = problems.base_problem(256, 256, 257)
    sim = lib.Sim(prm)
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lib.GrmhdError) as e:
        lib.grmhd_divb_noalloc(sim.ctx, dummy)
    assert e.value.status == lib.GRMHD_EINVAL
    assert "65536" in str(e.value)
    sim.close()
    # a context that fits still works afterwards
    prm2, P2, _ = fields.sine_box(16, 8, 4, ((1, 1, 1.0, 0),))
    s2 = lib.Sim(prm2)
    P = s2.to_device(P2)
    assert lib.grmhd_divb_noalloc(s2.ctx, P) == lib.grmhd_divb(s2.ctx, P)
    s2.close()
