"""Event timing of kernel launches through the C ABI: the class mask decides
which launches are bracketed, and timing leaves every result unchanged."""

import numpy as np
import pytest

import problems

pytestmark = pytest.mark.gpu


def test_profile_mask_times_only_the_chosen_classes(lib):
    prm, P0 = problems.fm_torus(n1=40, n2=16, n3=4)
    sim = lib.Sim(prm)
    P = sim.to_device(P0)
    Q = sim.to_device(P0)
    dt0 = sim.get_dt(P)
    dt_plain = sim.run(Q, 3, dt0)

    lib.grmhd_profile_kernels(sim.ctx, ["update"])
    lib.grmhd_profile(sim.ctx, True)
    dt_prof = sim.run(P, 3, dt0)
    lib.grmhd_profile(sim.ctx, False)
    ms, n = lib.grmhd_profile_read(sim.ctx, "update")
    assert n == 6 and ms > 0.0
    for name in ("ghosts", "sweeps", "fixup", "electrons"):
        assert lib.grmhd_profile_read(sim.ctx, name) == (0.0, 0)
    assert dt_prof == dt_plain
    assert np.array_equal(sim.to_host(P), sim.to_host(Q))

    # every class again (grmhd_profile(ctx, 1) clears the record)
    lib.grmhd_profile_kernels(sim.ctx, list(lib.KERNELS))
    lib.grmhd_profile(sim.ctx, True)
    sim.run(P, 1, dt_prof)
    lib.grmhd_profile(sim.ctx, False)
    counts = {name: lib.grmhd_profile_read(sim.ctx, name)[1] for name in ("ghosts", "sweeps", "update", "fixup")}
    assert counts == {"ghosts": 2, "sweeps": 2, "update": 2, "fixup": 2}

    for bad in (0, -1, 1 << lib.KERNELS["electrons"] + 1):
        assert lib.lib.grmhd_profile_kernels(sim.ctx, bad) == lib.GRMHD_EINVAL
    sim.close()
