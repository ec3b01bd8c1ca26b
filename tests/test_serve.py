"""Serving loop host logic on the CPU with a fake engine on a virtual clock:
exact step counts, admission in arrival order under the byte budget, memory
reuse, and latencies that match hand-computed queueing on toy streams."""

import numpy as np
import pytest

from problems.workloads import JobSpec, many_jobs, poisson_stream, BOX_N, KERR_N1, KERR_N2, KERR_N3
from paper_2110_10191_amd.serve import FakeEngine, Server, VirtualClock, percentile


def fake_state(spec):
    prm = dict(n1=spec.n1, n2=spec.n2, n3=spec.n3)
    return prm, None


def serve(specs, budget, quantum=25, rate=1e9, bytes_per_zone=1, overhead=0.0, fail_at=None):
    clock = VirtualClock()
    eng = FakeEngine(clock, rate=rate, bytes_per_zone=bytes_per_zone, overhead=overhead, fail_at=fail_at)
    srv = Server(eng, fake_state, budget, clock=clock, quantum=quantum, keep=[s.id for s in specs])
    rep = srv.run(specs)
    return rep, eng, srv


def test_two_jobs_one_slot_queue_behind_each_other():
    # 1e6 zones x 100 steps at 1e9 zone-cycles/s = 0.1 s each; budget holds one
    specs = [JobSpec(0, "box", 100, 100, 100, steps=100), JobSpec(1, "box", 100, 100, 100, steps=100)]
    rep, eng, _ = serve(specs, budget=1_000_000)
    lat = dict(zip([r.spec.id for r in rep.recs], rep.latency))
    assert lat[0] == pytest.approx(0.1)
    assert lat[1] == pytest.approx(0.2)
    assert rep.wait[1] == pytest.approx(0.1)
    assert rep.summary()["zone_cycles_per_s"] == pytest.approx(1e9)


def test_two_jobs_that_fit_run_together():
    specs = [JobSpec(0, "box", 100, 100, 100, steps=100), JobSpec(1, "box", 100, 100, 100, steps=100)]
    rep, eng, srv = serve(specs, budget=2_000_000)
    assert rep.latency == pytest.approx([0.2, 0.2])
    assert srv.max_running == 2


def test_idle_gap_and_exact_steps_with_uneven_counts():
    specs = [JobSpec(0, "box", 10, 10, 10, steps=30, arrival=0.0),
             JobSpec(1, "box", 10, 10, 10, steps=100, arrival=0.0),
             JobSpec(2, "box", 10, 10, 10, steps=7, arrival=5.0)]
    rep, eng, _ = serve(specs, budget=10**9, quantum=25)
    assert eng.steps == {0: 30, 1: 100, 2: 7}
    res = rep.results()
    assert res[2] == ("state", 2, 7)
    # cycle lengths: min(quantum, fewest steps left)
    assert [n for _, n in eng.cycles[:4]] == [25, 5, 25, 25]
    lat = dict(zip([r.spec.id for r in rep.recs], rep.latency))
    assert lat[2] == pytest.approx(7 * 1000 / 1e9)       # served alone after the gap


def test_budget_is_never_exceeded_and_order_is_fifo():
    specs = poisson_stream(60, lam=50.0, seed=7, steps=(20, 200))
    budget = 3 * max(s.zones for s in specs)
    rep, eng, srv = serve(specs, budget=budget, quantum=10, rate=5e8)
    assert srv.peak_in_use <= budget
    assert eng.steps == {s.id: s.steps for s in specs}
    admitted = [r.admitted for r in rep.recs]              # records are in arrival order
    assert all(b >= a for a, b in zip(admitted, admitted[1:]))
    for cyc, _ in eng.cycles:
        assert sum(specs[j].zones for j in cyc) <= budget
    s = rep.summary()
    assert s["completed"] == 60 and s["rejected"] == 0
    assert s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_oversized_job_is_rejected_not_hung():
    specs = [JobSpec(0, "box", 100, 100, 100, steps=5), JobSpec(1, "box", 10, 10, 10, steps=5)]
    rep, eng, _ = serve(specs, budget=10_000)
    assert [r.spec.id for r in rep.rejected] == [0]
    assert eng.steps == {1: 5}


def test_a_job_that_cannot_start_is_failed_and_frees_nothing():
    specs = [JobSpec(0, "box", 100, 100, 100, steps=100), JobSpec(1, "box", 100, 100, 100, steps=100),
             JobSpec(2, "box", 100, 100, 100, steps=100)]
    rep, eng, srv = serve(specs, budget=1_000_000, fail_at={1: -1})
    assert rep.failed == [1] and "Courant" in rep.errors[1]
    assert eng.steps == {0: 100, 2: 100}
    # job 1 is tried when job 0 frees the budget, fails at once and takes no
    # time: job 2 follows job 0 directly
    lat = {r.spec.id: r.done - r.spec.arrival for r in rep.recs}
    assert lat[0] == pytest.approx(0.1) and lat[1] == pytest.approx(0.1) and lat[2] == pytest.approx(0.2)
    s = rep.summary()
    assert s["completed"] == 2 and s["failed"] == 1
    assert s["zone_cycles_per_s"] == pytest.approx(1e9)
    assert srv.in_use == 0


def test_a_job_that_goes_non_finite_is_retired_at_once():
    # job 0 reports a non-finite speed from step 10 on; cycles are 4 steps, so
    # it is retired after the cycle that reaches step 12, not after 100 steps
    specs = [JobSpec(0, "box", 10, 10, 10, steps=100), JobSpec(1, "box", 10, 10, 10, steps=20)]
    rep, eng, srv = serve(specs, budget=10**9, quantum=4, fail_at={0: 10})
    res = rep.results()
    assert res[0] == ("state", 0, 12) and res[1] == ("state", 1, 20)
    assert rep.failed == [0] and rep.errors[0] == "non-finite signal speed"
    assert rep.summary()["completed"] == 1 and srv.in_use == 0


def test_percentile_is_nearest_rank():
    v = list(range(1, 101))
    assert percentile(v, 50) == 50
    assert percentile(v, 99) == 99
    assert percentile(v, 100) == 100
    assert percentile([3.0], 99) == 3.0
    assert np.isnan(percentile([], 50))


def test_stream_and_mix_generators():
    st = poisson_stream(300, lam=20.0, seed=4)
    gaps = np.diff([0.0] + [s.arrival for s in st])
    assert abs(gaps.mean() - 1 / 20.0) < 0.2 / 20.0
    assert all(200 <= s.steps <= 2000 for s in st)
    assert {s.kind for s in st} == {"torus", "bondi"}
    assert all(s.n1 in KERR_N1 and s.n2 in KERR_N2 and s.n3 in KERR_N3 and 0 <= s.a < 0.99 for s in st)
    assert poisson_stream(300, seed=4) == st                      # seeded
    mix = many_jobs()
    assert [s.kind for s in mix] == ["box"] * 32 + ["bondi"] * 32
    assert all(s.n1 == s.n2 == s.n3 and s.n1 in BOX_N for s in mix[:32])
    assert 20e6 < sum(s.zones for s in mix) < 40e6
