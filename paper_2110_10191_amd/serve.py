"""Continuous-batching server for many independent GRMHD problems on one GPU.

Jobs arrive over time, each with its own grid, initial state and number of
steps. The server admits arrived jobs in arrival order while their device
memory (context plus state, ``grmhd_context_bytes``) fits a budget, advances
every admitted job together through the library's batch calls (one grid per
kernel phase over all jobs, one step captured in a HIP graph and replayed),
retires each job after exactly its number of steps and reuses its memory for
the next arrivals. Membership changes only between replays: a cycle advances
all running jobs by min(quantum, fewest steps any of them has left).

Each job keeps its own time step on the device (the batch's per-job
dt <- min(cfl / sum_d ctop_d/dx_d, 1.3 dt) rule), carried bit-for-bit across
the batch re-creation that a membership change causes, so a job's result is
the same as when it runs alone.

Latency of a job = completion - arrival (queueing included); the report gives
p50/p99 latency and wait, throughput in zone-cycles/s over the makespan, and
the offered load.

    python -m paper_2110_10191_amd.serve [--jobs 300] [--lam 20] [--budget-gb 200]
"""

import argparse
import json
import math
import time
from collections import deque

import numpy as np


# ----------------------------------------------------------------- clocks

class RealClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def sleep_until(self, t):
        dt = t - self.now()
        if dt > 0:
            time.sleep(dt)


class VirtualClock:
    """Time that only moves when the engine or the scheduler says so."""

    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def advance(self, dt):
        self.t += dt

    def sleep_until(self, t):
        self.t = max(self.t, t)


# ----------------------------------------------------------------- engines

class JobFailed(RuntimeError):
    """A job the engine could not start (its initial state has no finite
    Courant step, or the library refused the problem)."""


class GpuEngine:
    """Runs admitted jobs as one batch of the HIP library (same recon and
    precision for every job)."""

    def __init__(self, recon, precision, device="cuda:0", tiles=None):
        import torch
        from . import _binding as B
        self.B = B
        self.torch = torch
        self.recon = recon
        self.precision = precision
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.tiles = tiles                  # {"sweep": (tx, ty), "update": (tx, ty)} or None
        self.jobs = {}                      # id -> [sim, state, dt, electrons (E, model, fel) or None]
        self.order = []                     # member ids of the current batch
        self.batch = None
        self.dirty = False

    def job_bytes(self, prm, electrons=False):
        """Device bytes of a job: context, state and, with electron heating, the
        entropies and their scratch (3 arrays of 2 doubles per padded zone)."""
        cb, sb = self.B.grmhd_context_bytes(prm)
        return cb + sb + (3 * sb // 4 if electrons else 0)

    def start(self, job_id, prm, P0, electrons=None):
        """electrons: None, or (E0, model, fel) for a job with electron heating
        (E0 the host entropies [2, n3+6, n2+6, n1+6])."""
        if prm["recon"] != self.recon or prm["precision"] != self.precision:
            raise ValueError("every job of the engine needs its recon and precision")
        sim = None
        try:
            with self.torch.cuda.device(self.device), self.torch.cuda.stream(self.stream):
                sim = self.B.Sim(prm, device=self.device, stream=self.stream)
                if self.tiles:
                    sim.set_tiles("sweep", *self.tiles["sweep"])
                    sim.set_tiles("update", *self.tiles["update"])
                P = sim.to_device(P0)
                dt = sim.get_dt(P)
                el = None
                if electrons is not None:
                    E0, model, fel = electrons
                    el = (sim.to_device(E0), model, fel)
        except self.B.GrmhdError as e:
            if sim is not None:
                sim.close()
            raise JobFailed(str(e)) from e
        self.jobs[job_id] = [sim, P, dt, el]
        self.dirty = True

    def _harvest_dt(self):
        """Copy the batch's per-job dt back to the job table (synchronises)."""
        if self.batch is None:
            return None
        dts, status = self.batch.get()
        for jid, dt, st in zip(self.order, dts, status):
            if jid in self.jobs:
                self.jobs[jid][2] = dt
        return dict(zip(self.order, status))

    def _rebuild(self):
        self._harvest_dt()
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        self.order = sorted(self.jobs)
        if self.order:
            sims = [self.jobs[j][0] for j in self.order]
            self.batch = self.B.Batch(sims, stream=self.stream)
            self.batch.set_dt([self.jobs[j][2] for j in self.order])
        self.dirty = False

    def advance(self, nsteps):
        """Enqueue nsteps steps of every running job (asynchronous)."""
        if self.dirty:
            self._rebuild()
        if self.batch is not None and nsteps > 0:
            els = [self.jobs[j][3] for j in self.order]
            self.batch.step([self.jobs[j][1] for j in self.order], nsteps=nsteps,
                            electrons=els if any(e is not None for e in els) else None)

    def sync(self):
        self.stream.synchronize()

    def status(self):
        """{id: 1 if the job's signal speeds went non-finite}; synchronises."""
        st = self._harvest_dt() or {}
        return {j: st.get(j, 0) for j in self.jobs}

    def finish(self, job_id, keep=False):
        """Retire a job; returns its final host state when keep is set (with
        electron heating, the pair (P, E))."""
        if job_id in self.order:
            self._harvest_dt()
        sim, P, _, el = self.jobs.pop(job_id)
        out = None
        if keep:
            with self.torch.cuda.stream(self.stream):
                out = sim.to_host(P) if el is None else (sim.to_host(P), sim.to_host(el[0]))
        self.dirty = True
        if self.batch is not None:
            # the batch holds the job's context: drop it before the context
            self.batch.close()
            self.batch = None
            self.order = []
        sim.close()
        return out


class FakeEngine:
    """Same interface, no device: a step of a job costs zones / rate seconds of
    a virtual clock. For testing the scheduler."""

    def __init__(self, clock, rate=1e9, bytes_per_zone=200, overhead=0.0, fail_at=None):
        self.clock = clock
        self.fail_at = dict(fail_at or {})   # job id -> step count from which its status is 1
                                             # (-1: the job cannot start)
        self.rate = rate
        self.bytes_per_zone = bytes_per_zone
        self.overhead = overhead
        self.jobs = {}
        self.pending = 0.0
        self.steps = {}
        self.cycles = []

    def job_bytes(self, prm, electrons=False):
        return prm["n1"] * prm["n2"] * prm["n3"] * self.bytes_per_zone

    def start(self, job_id, prm, P0, electrons=None):
        if self.fail_at.get(job_id) == -1:
            raise JobFailed(f"job {job_id}: no finite Courant step")
        self.jobs[job_id] = prm
        self.steps[job_id] = 0

    def advance(self, nsteps):
        zones = sum(p["n1"] * p["n2"] * p["n3"] for p in self.jobs.values())
        self.pending += zones * nsteps / self.rate + self.overhead
        for j in self.jobs:
            self.steps[j] += nsteps
        self.cycles.append((sorted(self.jobs), nsteps))

    def sync(self):
        self.clock.advance(self.pending)
        self.pending = 0.0

    def status(self):
        return {j: int(j in self.fail_at and self.steps[j] >= self.fail_at[j]) for j in self.jobs}

    def finish(self, job_id, keep=False):
        self.jobs.pop(job_id)
        return ("state", job_id, self.steps[job_id]) if keep else None


# ----------------------------------------------------------------- scheduler

class Record:
    __slots__ = ("spec", "prm", "state", "bytes", "admitted", "done", "left", "failed", "result", "error")

    def __init__(self, spec):
        self.spec = spec
        self.prm = None
        self.state = None
        self.bytes = 0
        self.admitted = None
        self.done = None
        self.left = spec.steps
        self.failed = False
        self.result = None
        self.error = None


def percentile(values, q):
    """Nearest-rank percentile: the smallest value with at least q% of the
    sample at or below it."""
    v = sorted(values)
    if not v:
        return float("nan")
    k = max(1, math.ceil(q / 100.0 * len(v)))
    return v[k - 1]


class Server:
    """Admission in arrival order under a byte budget, continuous batching.

    make_state(spec) -> (prm, P0), or (prm, P0, electrons) with electrons None
    or (E0, model, fel) for electron heating, places a job's initial data on
    the host; it runs while the device works on the previous cycle, for at
    most ``prefetch`` arrived jobs ahead of admission.
    """

    def __init__(self, engine, make_state, budget_bytes, clock=None, quantum=25, prefetch=8,
                 keep=(), progress=None):
        self.engine = engine
        self.make_state = make_state
        self.budget = budget_bytes
        self.clock = clock or RealClock()
        self.quantum = max(1, int(quantum))
        self.prefetch = max(1, int(prefetch))
        self.keep = set(keep)
        self.progress = progress            # progress(server, now, running, queued, done) per cycle
        self.in_use = 0
        self.peak_in_use = 0
        self.max_running = 0
        self.cycles = 0

    def _prepare(self, queue):
        n = 0
        for r in queue:
            if n >= self.prefetch:
                break
            if r.prm is None:
                made = self.make_state(r.spec)
                r.prm, r.state = made[0], tuple(made[1:])
                r.bytes = self.engine.job_bytes(r.prm, electrons=len(r.state) > 1 and r.state[1] is not None)
            n += 1

    def run(self, specs):
        recs = [Record(s) for s in sorted(specs, key=lambda s: (s.arrival, s.id))]
        future = deque(recs)
        queue = deque()
        running = {}
        rejected = []
        while future or queue or running:
            now = self.clock.now()
            while future and future[0].spec.arrival <= now:
                queue.append(future.popleft())
            self._prepare(queue)
            # admit in arrival order while the head fits
            while queue and queue[0].prm is not None:
                r = queue[0]
                if r.bytes > self.budget:
                    queue.popleft()
                    r.failed = True
                    r.done = now
                    rejected.append(r)
                    continue
                if self.in_use + r.bytes > self.budget:
                    break
                queue.popleft()
                try:
                    self.engine.start(r.spec.id, r.prm, *r.state)
                except JobFailed as e:
                    # retired at once; the other jobs never see it
                    r.state = None
                    r.admitted = r.done = self.clock.now()
                    r.failed = True
                    r.error = str(e)
                    continue
                r.state = None
                r.admitted = self.clock.now()
                self.in_use += r.bytes
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                running[r.spec.id] = r
                r.left = max(0, r.left)
                self._prepare(queue)
            if not running:
                if future and not queue:
                    self.clock.sleep_until(future[0].spec.arrival)
                continue
            self.max_running = max(self.max_running, len(running))
            n = min(self.quantum, min(r.left for r in running.values()))
            self.engine.advance(n)
            # host work for the next admissions overlaps the device
            now = self.clock.now()
            while future and future[0].spec.arrival <= now:
                queue.append(future.popleft())
            self._prepare(queue)
            self.engine.sync()
            self.cycles += 1
            now = self.clock.now()
            for r in running.values():
                r.left -= n
            # a job whose signal speeds went non-finite is retired now, with
            # an error, instead of running out its step count
            status = self.engine.status()
            finished = [r for r in running.values() if r.left <= 0 or status.get(r.spec.id, 0)]
            for r in finished:
                if status.get(r.spec.id, 0):
                    r.failed = True
                    r.error = "non-finite signal speed"
                r.result = self.engine.finish(r.spec.id, keep=r.spec.id in self.keep)
                r.done = now
                self.in_use -= r.bytes
                del running[r.spec.id]
            if self.progress:
                self.progress(self, now, len(running), len(queue),
                              sum(1 for r in recs if r.done is not None))
        return Report(recs, rejected, self)


class Report:
    def __init__(self, recs, rejected, server):
        self.recs = recs
        self.rejected = rejected
        done = [r for r in recs if r.admitted is not None]
        ok = [r for r in done if not r.failed]
        # latency, wait and work of the jobs that completed (ok order)
        self.latency = [r.done - r.spec.arrival for r in ok]
        self.wait = [r.admitted - r.spec.arrival for r in ok]
        self.work = sum(r.spec.zones * r.spec.steps for r in ok)
        t_first = min((r.spec.arrival for r in recs), default=0.0)
        t_last = max((r.done for r in done), default=0.0)
        self.makespan = t_last - t_first if done else 0.0
        self.failed = [r.spec.id for r in done if r.failed]
        self.errors = {r.spec.id: r.error for r in done if r.failed}
        self.server = server

    def results(self):
        return {r.spec.id: r.result for r in self.recs if r.result is not None}

    def summary(self):
        n = len(self.recs)
        span = max((r.spec.arrival for r in self.recs), default=0.0)
        lam = (n - 1) / span if n > 1 and span > 0 else float("nan")
        mean_work = np.mean([r.spec.zones * r.spec.steps for r in self.recs]) if n else 0.0
        return {
            "jobs": n,
            "completed": len(self.latency),
            "rejected": len(self.rejected),
            "failed": len(self.failed),
            "p50_latency_s": percentile(self.latency, 50),
            "p99_latency_s": percentile(self.latency, 99),
            "p50_wait_s": percentile(self.wait, 50),
            "p99_wait_s": percentile(self.wait, 99),
            "makespan_s": self.makespan,
            "zone_cycles_per_s": self.work / self.makespan if self.makespan > 0 else float("nan"),
            "offered_zone_cycles_per_s": float(lam * mean_work),
            "cycles": self.server.cycles,
            "max_running": self.server.max_running,
            "peak_bytes": self.server.peak_in_use,
        }


# ----------------------------------------------------------------- command line

def _where_unequal(a, b):
    """Count, largest difference and first indices of the entries of two
    same-shape arrays that are not bitwise equal (NaN counts as unequal)."""
    w = np.argwhere(~(a == b))
    d = np.abs(a - b)
    return {"count": int(len(w)), "max_abs": float(np.nanmax(d)) if d.size else 0.0, "first": w[:8].tolist()}


def identity_check(report, specs, make_state, recon, precision, sample, device="cuda:0", tiles=None, diffs=None):
    """Re-run each sampled job alone and compare its final state bit for bit
    with the state it reached inside the mix. diffs: a dict that receives, per
    job that differs, where its arrays differ."""
    results = report.results()
    by_id = {s.id: s for s in specs}
    out = {}
    for jid in sample:
        if jid not in results:
            continue
        spec = by_id[jid]
        eng = GpuEngine(recon, precision, device=device, tiles=tiles)
        made = make_state(spec)
        eng.start(jid, *made)
        eng.advance(spec.steps)
        eng.sync()
        alone = eng.finish(jid, keep=True)
        mixed = results[jid]
        if isinstance(alone, tuple):
            out[jid] = isinstance(mixed, tuple) and all(np.array_equal(a, b) for a, b in zip(alone, mixed))
        else:
            out[jid] = bool(np.array_equal(alone, mixed))
        if not out[jid] and diffs is not None:
            pairs = zip(alone, mixed) if isinstance(alone, tuple) and isinstance(mixed, tuple) else [(alone, mixed)]
            diffs[jid] = [_where_unequal(np.asarray(a), np.asarray(b)) for a, b in pairs
                          if np.shape(a) == np.shape(b)]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--jobs", type=int, default=300)
    ap.add_argument("--lam", type=float, default=20.0)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--quantum", type=int, default=25)
    ap.add_argument("--recon", choices=["mc", "weno5"], default="weno5")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--min-steps", type=int, default=200)
    ap.add_argument("--max-steps", type=int, default=2000)
    ap.add_argument("--identity", type=int, default=8, help="jobs re-run alone for the identity check")
    ap.add_argument("--tune", action="store_true", help="autotune tiles on the first job's grid")
    ap.add_argument("--electrons", choices=["constant", "kawazura", "werner", "rowan", "howes", "sharma"],
                    default=None, help="evolve the torus jobs with electron heating by this model")
    args = ap.parse_args(argv)

    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import problems
    from problems.workloads import poisson_stream

    recon = problems.RECON_WENO5 if args.recon == "weno5" else problems.RECON_MC
    precision = problems.MIXED if args.precision == "mixed" else problems.FP64
    specs = poisson_stream(args.jobs, args.lam, args.seed, steps=(args.min_steps, args.max_steps))

    def make_state(spec):
        prm, P0 = spec.make(recon=recon, precision=precision)
        if args.electrons and spec.kind == "torus":
            return prm, P0, (problems.electron_scalars(P0, prm["gam"]), args.electrons, 0.5)
        return prm, P0

    tiles = None
    if args.tune:
        from . import tune
        prm, P0 = make_state(max(specs, key=lambda s: s.zones))[:2]
        tiles = tune.tune_problem(prm, P0)
    rng = np.random.default_rng(args.seed + 1000)
    sample = sorted(int(x) for x in rng.choice(len(specs), size=min(args.identity, len(specs)), replace=False))
    eng = GpuEngine(recon, precision, tiles=tiles)
    last = [0.0]

    def progress(srv, now, running, queued, done):
        if now - last[0] >= 5.0:
            last[0] = now
            print(f"[serve] t={now:.1f}s done={done} running={running} queued={queued} "
                  f"cycles={srv.cycles} bytes={srv.in_use / 1e9:.1f}GB", file=sys.stderr, flush=True)

    srv = Server(eng, make_state, int(args.budget_gb * 1e9), quantum=args.quantum, keep=sample,
                 progress=progress)
    rep = srv.run(specs)
    summ = rep.summary()
    print(f"[serve] stream done in {rep.makespan:.1f}s; identity check of {len(sample)} jobs",
          file=sys.stderr, flush=True)
    ident = identity_check(rep, specs, make_state, recon, precision, sample, tiles=tiles)
    summ["identity_alone_vs_mix"] = {str(k): v for k, v in ident.items()}
    summ["config"] = {"workload": f"poisson stream of {args.jobs} torus/Bondi jobs",
                      "lam_per_s": args.lam, "seed": args.seed, "budget_gb": args.budget_gb,
                      "recon": args.recon, "precision": args.precision, "quantum": args.quantum,
                      "steps": [args.min_steps, args.max_steps], "tiles": tiles,
                      "electrons": args.electrons}
    print(json.dumps(summ), flush=True)
    return 0 if all(ident.values()) and not rep.failed else 1


if __name__ == "__main__":
    raise SystemExit(main())
