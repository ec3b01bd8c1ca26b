"""Serving on the device: a short stream of uneven torus and Bondi jobs,
admitted as they arrive and retired after exactly their step counts, with
batch re-creation at every membership change; each job's final state equals,
bit for bit, the state it reaches when run alone."""

import numpy as np
import pytest

import problems
from problems.workloads import JobSpec
from paper_2110_10191_amd.serve import GpuEngine, Server, identity_check

pytestmark = pytest.mark.gpu


def make_state(recon, precision):
    def mk(spec):
        return spec.make(recon=recon, precision=precision)
    return mk


@pytest.mark.parametrize("recon,precision", [(problems.RECON_MC, problems.FP64),
                                             (problems.RECON_WENO5, problems.MIXED)],
                         ids=["mc_fp64", "weno5_mixed"])
def test_stream_matches_jobs_run_alone(lib, recon, precision):
    specs = [
        JobSpec(0, "torus", 48, 32, 8, a=0.9, steps=9, arrival=0.0),
        JobSpec(1, "bondi", 40, 24, 4, a=0.3, steps=5, arrival=0.0),
        JobSpec(2, "torus", 64, 20, 6, a=0.5, steps=12, arrival=0.05),
        JobSpec(3, "bondi", 36, 30, 3, a=0.0, steps=3, arrival=0.1),
        JobSpec(4, "box", 16, 16, 16, steps=7, arrival=0.1),
        JobSpec(5, "torus", 32, 24, 4, a=0.98, steps=6, arrival=0.3),
    ]
    mk = make_state(recon, precision)
    eng = GpuEngine(recon, precision)
    # the budget holds about three of the jobs at once
    sizes = sorted(eng.job_bytes(mk(s)[0]) for s in specs)
    budget = sum(sizes[-3:])
    srv = Server(eng, mk, budget, quantum=4, keep=[s.id for s in specs])
    rep = srv.run(specs)
    summ = rep.summary()
    assert summ["completed"] == len(specs) and summ["failed"] == 0 and summ["rejected"] == 0
    assert srv.peak_in_use <= budget
    assert summ["p99_latency_s"] >= summ["p50_latency_s"] > 0
    assert srv.cycles >= 4
    diffs = {}
    ident = identity_check(rep, specs, mk, recon, precision, [s.id for s in specs], diffs=diffs)
    assert ident == {s.id: True for s in specs}, diffs


def test_a_job_that_cannot_start_is_failed_and_the_others_are_untouched(lib):
    """Fault injection: a job whose initial state holds a NaN has no finite
    Courant step; the server retires it at admission with the library's error
    and every other job still ends bit for bit as when run alone."""
    specs = [
        JobSpec(0, "torus", 48, 32, 8, a=0.9, steps=6, arrival=0.0),
        JobSpec(1, "bondi", 40, 24, 4, a=0.3, steps=5, arrival=0.0),
        JobSpec(2, "torus", 32, 24, 4, a=0.5, steps=4, arrival=0.0),
    ]
    clean = make_state(problems.RECON_MC, problems.FP64)

    def mk(spec):
        prm, P0 = clean(spec)
        if spec.id == 1:
            P0 = P0.copy()
            P0[1, 4, 8, 12] = np.nan
        return prm, P0

    eng = GpuEngine(problems.RECON_MC, problems.FP64)
    srv = Server(eng, mk, 1 << 40, quantum=2, keep=[0, 2])
    rep = srv.run(specs)
    assert rep.failed == [1] and "status -5" in rep.errors[1]
    assert rep.summary()["completed"] == 2 and srv.in_use == 0
    ident = identity_check(rep, specs, clean, problems.RECON_MC, problems.FP64, [0, 2])
    assert ident == {0: True, 2: True}


def test_stream_with_electron_heating_matches_jobs_run_alone(lib):
    """Jobs with electron heating (two models) and without share the served
    batch; every job's final primitives and entropies equal, bit for bit, the
    ones it reaches alone."""
    specs = [
        JobSpec(0, "torus", 48, 32, 8, a=0.9, steps=7, arrival=0.0),
        JobSpec(1, "bondi", 40, 24, 4, a=0.3, steps=5, arrival=0.0),
        JobSpec(2, "torus", 64, 20, 6, a=0.5, steps=9, arrival=0.05),
        JobSpec(3, "box", 16, 16, 16, steps=6, arrival=0.1),
    ]
    heat = {0: ("howes", 0.0), 3: ("constant", 0.4)}
    clean = make_state(problems.RECON_MC, problems.FP64)

    def mk(spec):
        prm, P0 = clean(spec)
        if spec.id in heat:
            return prm, P0, (problems.electron_scalars(P0, prm["gam"], te_ti=0.5),) + heat[spec.id]
        return prm, P0

    eng = GpuEngine(problems.RECON_MC, problems.FP64)
    srv = Server(eng, mk, 1 << 40, quantum=3, keep=[s.id for s in specs])
    rep = srv.run(specs)
    assert rep.summary()["completed"] == 4 and not rep.failed
    res = rep.results()
    assert isinstance(res[0], tuple) and isinstance(res[3], tuple) and not isinstance(res[1], tuple)
    diffs = {}
    ident = identity_check(rep, specs, mk, problems.RECON_MC, problems.FP64, [s.id for s in specs], diffs=diffs)
    assert ident == {s.id: True for s in specs}, diffs


def test_tuned_tiles_do_not_change_a_served_job(lib):
    spec = JobSpec(0, "torus", 48, 32, 8, a=0.9, steps=4)
    mk = make_state(problems.RECON_MC, problems.FP64)
    outs = []
    for tiles in (None, {"sweep": (128, 2), "update": (32, 8)}):
        eng = GpuEngine(problems.RECON_MC, problems.FP64, tiles=tiles)
        prm, P0 = mk(spec)
        eng.start(0, prm, P0)
        eng.advance(2)
        eng.advance(2)
        eng.sync()
        outs.append(eng.finish(0, keep=True))
    assert np.array_equal(outs[0], outs[1])
