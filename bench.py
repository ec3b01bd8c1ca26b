#!/usr/bin/env python3
"""Throughput of the GRMHD zone update on one MI355X.

    python bench.py [--steps K] [--warmup W] [--precision fp64|mixed] [--recon mc|weno5]

Workload (default): the Fishbone-Moncrief torus in Kerr (a = 0.9375, r_in = 6,
r_max = 12, gamma = 13/9) on a 288 x 128 x 128 funky-MKS grid to r = 1000,
single-loop field at beta = 100, seeded 4 % noise on u; MC reconstruction,
LLF fluxes, Flux-CT, predictor-corrector, FP64. Synthetic initial data from
``problems.fm_torus``; the state is resident in HBM before timing starts.

A step is one full predictor-corrector cycle of every zone, including the
Courant step for the next one (dt <- min(dt_next, 1.3 dt)). By default the
steps go through grmhd_run, which keeps the step size on the device so the
host does not wait between steps (``--path host`` calls grmhd_step once a
step and reads dt back each time; the two give identical states). The metric is
zone-cycles per second: interior zones x steps / wall seconds over the timed
steps (bracketed by device synchronisation), which run as 5 consecutive
repeats whose median rate is reported beside the total. Kernel durations over
the same timed region come from HIP events the library records on its stream
around every launch. The roofline fraction is the dominant kernel's
algorithmic bytes per launch over its mean duration against 8 TB/s, where the
algorithmic bytes are the method's compulsory bytes (the P^n, P_h, P^n+1
state traffic of a step plus the 2D geometry, 338.75 B per zone-cycle on the
benchmark torus) for the zone-cycles one launch advances; this design's own
byte model (face fluxes included) is a separate view. The line also carries a
few steps of the 64-job batched workload against the per-job FP64 loop
(``many``), the serving loop's p50 / p99 job latency on a short Poisson stream
of uneven jobs (``serving``), and the oracle (NumPy FP64, one core) timed on a
bounded sample of the same torus.

``--coords cks`` times another workload instead: a magnetised Michel flow on a
168^3 Cartesian Kerr-Schild box, whose geometry tables are 3D (every zone
reads its own connection: 992 B per zone-cycle compulsory in FP64, where
the metric is evaluated in closed form).

Prints one JSON line on stdout.
"""

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK = 8.0e12          # bytes/s, MI355X HBM3E
FP64_PEAK = 78.6e12        # flop/s, MI355X FP64 vector
FP32_PEAK = 157.3e12       # flop/s, MI355X FP32 vector
NG = 3
CKS = 3                    # Cartesian Kerr-Schild coordinates
TIMED_KERNELS = ["sweeps", "update"]  # event-timed inside the timed region


def compulsory_bytes_per_zone_cycle(prm):
    """The method's compulsory HBM bytes per zone-cycle with an FP64 state: a
    step reads P^n and writes P_h (predictor), reads P^n and P_h and writes
    P^{n+1} (corrector), 5 x 64 = 320 B a zone; plus, on a Kerr grid, the
    axisymmetric geometry, about 150 doubles per (x1, x2) column per substep,
    shared by the n3 zones of the column. 338.75 B on the 288 x 128 x 128 torus.
    Cartesian Kerr-Schild geometry depends on x3, so every zone reads its own
    connection (40 values, by centred differences) and floor scales (2) each
    substep; the metric, its inverse, sqrt(-g) and the lapse have closed
    forms that the kernels evaluate instead of reading (the update at the
    centre; the FP64 face-flux pass at the faces, while the mixed-precision
    one reads the float face tables, 3 x 22 values)."""
    if prm["coords"] == CKS:
        faces = 3 * 22 * 4 if prm["precision"] == 1 else 0
        return 320.0 + 2 * (42 * 8 + faces)
    geo = 0.0 if prm["coords"] == 0 else 2 * 150 * 8 / prm["n3"]
    return 320.0 + geo


def split_design_bytes(kernel, prm, mixed):
    """Bytes one launch of this split design moves at minimum: every value it
    reads once and every value it writes once (stencil re-reads are cache
    traffic), including the face fluxes the sweeps write and the update reads
    back. A view of the design, not of the method: the method's compulsory
    bytes are compulsory_bytes_per_zone_cycle."""
    n1, n2, n3 = prm["n1"], prm["n2"], prm["n3"]
    fb = 4 if mixed else 8
    recon_reach = 3 if prm["recon"] == 1 else 2          # zones below / above+1 a face
    if kernel == "sweeps":
        # the state over the stencil's reach around the faces, once; the 7
        # stored components of every face of the three directions; the three
        # 2D face tables once
        cells = (n1 + 2 * recon_reach) * (n2 + 2 * recon_reach) * (n3 + 2 * recon_reach)
        faces = ((n1 + 1) * (n2 + 2) * (n3 + 2) + (n1 + 2) * (n2 + 1) * (n3 + 2)
                 + (n1 + 2) * (n2 + 2) * (n3 + 1))
        geo = 3 * 22 * fb * (n1 + 2) * (n2 + 2) * ((n3 + 2) if prm["coords"] == CKS else 1)
        return 64 * cells + 7 * fb * faces + geo
    if kernel == "update":
        zones = n1 * n2 * n3
        # 7 flux components per direction (5 hydro + 2 transverse B); the states
        # read: one in the predictor (P_base = P_s = P), two in the corrector
        # (P, P_h), 96 B a zone on average over the two launches of a step;
        # P_out written; one flag byte; the 2D centre table once
        return zones * (21 * fb + 96 + 64 + 1) + 64 * 8 * n1 * n2 * (n3 if prm["coords"] == CKS else 1)
    raise KeyError(kernel)


def arithmetic_ceiling(flops_per_step, zones, per_zc, step_s):
    """The step's counted VALU work against its compulsory bytes.

    A step that does flops_per_step FP64 operations cannot take less than
    flops_per_step / FP64_PEAK seconds, so the compulsory bytes it moves
    (per_zc per zone) can reach at most this fraction of the HBM peak:
    (zones * per_zc / (flops_per_step / FP64_PEAK)) / HBM_PEAK, capped at 1.
    Where the method's FP64 operations per compulsory byte exceed the chip's
    balance (FP64_PEAK / HBM_PEAK, 9.8 flop/B) the step is bound by FP64
    issue, not by HBM, and the HBM fraction has that ceiling."""
    bytes_step = zones * per_zc
    t_min = flops_per_step / FP64_PEAK
    return {"fp64_flops_per_zone_cycle": flops_per_step / zones,
            "flop_per_compulsory_byte": flops_per_step / bytes_step,
            "machine_balance_flop_per_byte": FP64_PEAK / HBM_PEAK,
            "step_compulsory_frac_ceiling": min(1.0, bytes_step / t_min / HBM_PEAK) if t_min > 0 else 1.0,
            "step_fp64_frac": flops_per_step / step_s / FP64_PEAK}


def device_copy_bandwidth(torch, dev, gib=1.0, reps=5):
    """Best of a few plain device-to-device copies, bytes read + written per second."""
    nel = int(gib * 2 ** 30) // 8
    a = torch.ones(nel, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        t = e0.elapsed_time(e1) / 1e3
        best = t if best is None else min(best, t)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nel * 8 / best


def measured_traffic(workload):
    """HBM bytes per launch of each kernel class from the committed counter
    summary (profiles/hbm_traffic.json, per workload: FETCH_SIZE and
    WRITE_SIZE scaled by a plain copy), with launches per step, only while the
    library is the build those counters were taken on."""
    path = os.path.join(HERE, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        from paper_2110_10191_amd import tune
        if rec.get("library_hash") == tune.library_hash() and workload in rec.get("workloads", {}):
            return rec["workloads"][workload]["kernels"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def measured_flops(workload):
    """Per-kernel FP64 and FP32 VALU flops per launch from the committed counter
    summary (profiles/valu_flops.json: (2 FMA + ADD + MUL) x 64 lanes per
    precision), only while the library is the build they were taken on."""
    path = os.path.join(HERE, "profiles", "valu_flops.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        from paper_2110_10191_amd import tune
        if rec.get("library_hash") == tune.library_hash() and workload in rec.get("workloads", {}):
            return rec["workloads"][workload]
    except (OSError, ValueError, KeyError):
        pass
    return None


def cpu_baseline(prm_full, nslabs=32, nsteps=2):
    """The oracle on the same torus grid with nslabs x3 slabs, nsteps steps."""
    import oracle
    import problems
    prm, P0 = problems.fm_torus(n1=prm_full["n1"], n2=prm_full["n2"], n3=nslabs,
                                recon=prm_full["recon"])
    g = oracle.Grid(prm)
    dt = 0.005
    P = P0
    t0 = time.perf_counter()
    for _ in range(nsteps):
        P, _, _ = oracle.step(P, g, dt)
    secs = time.perf_counter() - t0
    zones = prm["n1"] * prm["n2"] * prm["n3"]
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {
        "value": zones * nsteps / secs,
        "unit": "zone-cycles/s",
        "cores": 1,
        "host_cpu": model,
        "host_os_cpu_count": os.cpu_count(),
        "kind": "oracle",
        "sample": (f"{nsteps} FP64 steps of the {prm['n1']}x{prm['n2']} FMKS torus grid with {nslabs} x3 slabs "
                   f"({zones} zones, same per-zone work as the benchmark grid) in {secs:.1f} s; "
                   "NumPy element-wise, single thread"),
    }


def cpu_baseline_cks(prm_full, nsteps=2):
    """The oracle on a 48^3 Cartesian Kerr-Schild box of the same flow."""
    import oracle
    import problems
    prm, P0 = problems.cks_bondi(48, 48, 48, recon=prm_full["recon"])
    g = oracle.Grid(prm)
    dt = oracle.get_dt(P0, g)
    P = P0
    t0 = time.perf_counter()
    for _ in range(nsteps):
        P, _, _ = oracle.step(P, g, dt)
    secs = time.perf_counter() - t0
    zones = 48 ** 3
    return {"value": zones * nsteps / secs, "unit": "zone-cycles/s", "cores": 1,
            "host_os_cpu_count": os.cpu_count(), "kind": "oracle",
            "sample": f"{nsteps} FP64 steps of a 48^3 Cartesian Kerr-Schild box of the same flow in {secs:.1f} s"}


def serving_record(n_jobs=48, lam=7.0, seed=4, steps=(100, 400), identity=2):
    """The serving loop (``paper_2110_10191_amd.serve``) on a short Poisson
    stream of torus and Kerr Bondi jobs of uneven grids (WENO5, mixed
    precision, continuous batching under a 200 GB budget): job latency from
    arrival to completion (p50 / p99), queueing wait, and zone-cycles/s over the
    makespan, with the offered rate for comparison; a few jobs are re-run
    alone and must be bitwise equal to their results in the mix."""
    import numpy as np
    import problems
    from problems.workloads import poisson_stream
    from paper_2110_10191_amd import serve
    recon, precision = problems.RECON_WENO5, problems.MIXED
    specs = poisson_stream(n_jobs, lam, seed, steps=steps)

    def make_state(spec):
        return spec.make(recon=recon, precision=precision)

    rng = np.random.default_rng(seed + 1000)
    sample = sorted(int(x) for x in rng.choice(len(specs), size=identity, replace=False))
    # batch tiles from the autotuner, timed on the stream's largest grid
    from paper_2110_10191_amd import tune
    t_tune = time.perf_counter()
    prm_big, P_big = make_state(max(specs, key=lambda sp: sp.zones))
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        tiles = tune.tune_problem(prm_big, P_big, cache=tune.TileCache(path=os.path.join(tmp, "tiles.json")),
                                  force=True, steps=2, repeats=2)
    t_tune = time.perf_counter() - t_tune
    eng = serve.GpuEngine(recon, precision, tiles=tiles)
    srv = serve.Server(eng, make_state, int(200e9), quantum=25, keep=sample)
    rep = srv.run(specs)
    summ = rep.summary()
    ident = serve.identity_check(rep, specs, make_state, recon, precision, sample, tiles=tiles)
    summ["identity_alone_vs_mix"] = {str(k): v for k, v in ident.items()}
    summ["config"] = {"workload": f"poisson stream of {n_jobs} torus / Kerr Bondi jobs (64-192 x 64-128 x 32-64)",
                      "lam_per_s": lam, "seed": seed, "steps": list(steps), "recon": "weno5",
                      "precision": "mixed", "budget_gb": 200.0, "quantum": 25,
                      "tiles": {k: list(v) for k, v in tiles.items()}, "tune_s": t_tune}
    return summ


def many_record(steps, warmup, tune_tiles):
    """64 independent uneven jobs (32 periodic boxes N^3, N in 32..96; 32 Bondi
    flows in Kerr, a ~ U[0, 0.99], up to 192 x 128 x 64): every job advanced
    by the batch calls (one grid per kernel phase over all jobs, a captured
    HIP graph per step, per-job dt on the device), in FP64 and in mixed
    precision, against the plain per-job FP64 loop: one job after another,
    each through grmhd_run (its step size kept on the device, one host
    synchronisation per job)."""
    import torch
    import paper_2110_10191_amd as g
    from paper_2110_10191_amd import tune
    import problems
    from problems.workloads import many_jobs

    specs = many_jobs(64, seed=3)
    zones = sum(s.zones for s in specs)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t_gen = time.perf_counter()
    init = [sp.make(recon=problems.RECON_MC, precision=problems.FP64) for sp in specs]
    print(f"[bench] many: {len(specs)} jobs, {zones} zones of initial data in "
          f"{time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
    res = {}
    for prec_name, prec in (("fp64", problems.FP64), ("mixed", problems.MIXED)):
        sims, states = [], []
        for prm, P0 in init:
            sim = g.Sim(dict(prm, precision=prec), device=dev)
            sims.append(sim)
            states.append(sim.to_device(P0))
        torch.cuda.synchronize()
        tiles = None
        if tune_tiles:
            t_tune = time.perf_counter()
            tiles, _ = tune.tune_batch(sims, states, steps=2, repeats=1)
            print(f"[bench] many {prec_name}: batch tiles {tiles} ({time.perf_counter() - t_tune:.1f} s)",
                  file=sys.stderr, flush=True)
        dts = [s.get_dt(P) for s, P in zip(sims, states)]
        b = g.Batch(sims)
        b.set_dt(dts)
        b.step(states, nsteps=warmup)
        b.get()
        t0 = time.perf_counter()
        b.step(states, nsteps=steps)
        _, status = b.get()
        secs = time.perf_counter() - t0
        b.close()
        res[f"batched_{prec_name}"] = {"value": zones * steps / secs, "ms_per_step": secs / steps * 1e3,
                                       "tiles": tiles, "bad_jobs": int(sum(status))}
        print(f"[bench] many batched {prec_name}: {zones * steps / secs:.3e} zone-cycles/s",
              file=sys.stderr, flush=True)
        if prec == problems.FP64:
            # the loop keeps each job's own default tiles (tuning applies to the batch)
            for s in sims:
                s.set_tiles("sweep", *tune.DEFAULT["sweep"])
                s.set_tiles("update", *tune.DEFAULT["update"])
            dts = [s.get_dt(P) for s, P in zip(sims, states)]
            dts = [s.run(P, 1, dt) for s, P, dt in zip(sims, states, dts)]    # warm each job's code path
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s, P, dt in zip(sims, states, dts):
                s.run(P, steps, dt)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            res["per_job_loop_fp64"] = {"value": zones * steps / secs, "ms_per_step": secs / steps * 1e3,
                                        "driver": "grmhd_run per job"}
            print(f"[bench] many per-job FP64 loop: {zones * steps / secs:.3e} zone-cycles/s",
                  file=sys.stderr, flush=True)
        for s in sims:
            s.close()
        del states
        torch.cuda.empty_cache()
    base = res["per_job_loop_fp64"]["value"]
    return {
        "workload": "64 uneven jobs: 32 boxes N^3 (N in 32..96), 32 Kerr Bondi (up to 192x128x64), MC, seed 3",
        "zones": zones, "steps": steps, "warmup": warmup,
        "batched_fp64": res["batched_fp64"],
        "batched_mixed": res["batched_mixed"],
        "per_job_loop_fp64": res["per_job_loop_fp64"],
        "speedup_batched_mixed_vs_loop": res["batched_mixed"]["value"] / base,
        "speedup_batched_fp64_vs_loop": res["batched_fp64"]["value"] / base,
    }


def bench_many(args):
    rec = many_record(args.steps, args.warmup, args.tune)
    out = {
        "metric": "zone-cycles/s, batched uneven jobs vs the per-job FP64 loop",
        "value": rec["batched_mixed"]["value"],
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rec["batched_mixed"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": rec["workload"], "zones": rec["zones"], "seed": 3},
        "many": rec,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--recon", choices=["mc", "weno5"], default="mc")
    ap.add_argument("--grid", type=int, nargs=3, default=None,
                    help="zones (default 288 128 128 for the torus, 168 168 168 for --coords cks)")
    ap.add_argument("--coords", choices=["fmks", "cks"], default="fmks",
                    help="fmks: the torus (default); cks: a magnetised Michel flow on a Cartesian "
                         "Kerr-Schild box (3D geometry tables), a workload of its own")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-many", action="store_true",
                    help="leave out the 64-job batched-vs-loop sub-record of the torus line")
    ap.add_argument("--many-steps", type=int, default=5, help="timed steps of the 64-job sub-record")
    ap.add_argument("--no-serving", action="store_true",
                    help="leave out the serving sub-record (p50/p99 job latency of a short Poisson stream)")
    ap.add_argument("--workload", choices=["torus", "many"], default="torus",
                    help="torus: one large torus (default); many: 64 uneven jobs batched vs looped")
    ap.add_argument("--tune", action="store_true", help="autotune the batch tiles (workload many)")
    ap.add_argument("--path", choices=["device", "host"], default="device",
                    help="device: grmhd_run, the step size kept on the device (default); host: one "
                         "grmhd_step per step with dt read back each step")
    ap.add_argument("--electrons", choices=["constant", "kawazura", "werner", "rowan", "howes", "sharma"], default=None,
                    help="step the electron entropies too (grmhd_run_electrons, or grmhd_step_electrons "
                         "with --path host) with this heating model (constant: f_e = 0.5)")
    ap.add_argument("--copy-calibration-gib", type=float, default=0.0,
                    help="also run one plain device copy of this size (for counter scaling)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library runs the zone update on a single device "
              "(multi-GPU block decomposition is a design note only). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "many":
        bench_many(args)
        return

    import torch
    import problems
    import paper_2110_10191_amd as g

    recon = problems.RECON_MC if args.recon == "mc" else problems.RECON_WENO5
    mixed = args.precision == "mixed"
    cks = args.coords == "cks"
    n1, n2, n3 = args.grid or ([168, 168, 168] if cks else [288, 128, 128])
    t_gen = time.perf_counter()
    prec = problems.MIXED if mixed else problems.FP64
    if cks:
        prm, P0 = problems.cks_bondi(n1, n2, n3, recon=recon, precision=prec)
    else:
        prm, P0 = problems.fm_torus(n1=n1, n2=n2, n3=n3, recon=recon, precision=prec)
    print(f"[bench] initial data {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sim = g.Sim(prm, device=dev)
    P = sim.to_device(P0)
    torch.cuda.synchronize()

    dt = sim.get_dt(P)
    E = None
    if args.electrons:
        E = sim.to_device(problems.electron_scalars(P0, prm["gam"]))

    def advance(nsteps, dt):
        """nsteps steps through the chosen driver; returns the next dt. Every
        driver synchronises the host with the device when it returns."""
        if args.path == "device":
            # grmhd_run(_electrons): the step size kept on the device (dt <-
            # min(dt_next, 1.3 dt), applied by the next step's first ghost-fill
            # launch); one sync at the end
            if E is not None:
                return sim.run_electrons(P, E, nsteps, dt, args.electrons)
            return sim.run(P, nsteps, dt)
        # one grmhd_step(_electrons) call per step, dt read back every step
        for _ in range(nsteps):
            dn = sim.step_electrons(P, E, dt, args.electrons) if E is not None else sim.step(P, dt)
            dt = min(dn, 1.3 * dt)
        return dt

    dt = advance(args.warmup, dt)
    torch.cuda.synchronize()
    print(f"[bench] warmup done, dt = {dt:.3e}", file=sys.stderr, flush=True)
    # exactly args.steps timed steps, in 5 consecutive repeats (or fewer when
    # there are fewer steps) so the median repeat rate comes with the total;
    # every launch of the two candidates for the dominant kernel (face fluxes,
    # update) is bracketed by library events on its stream. The other classes
    # run without events inside the timed region (each event record costs the
    # stream a few microseconds) and are timed in a short untimed pass after it.
    nrep = min(5, args.steps)
    reps = [args.steps // nrep + (1 if r < args.steps % nrep else 0) for r in range(nrep)]
    g.grmhd_profile_kernels(sim.ctx, TIMED_KERNELS)
    g.grmhd_profile(sim.ctx, True)
    torch.cuda.synchronize()
    rep_rates = []
    t0 = time.perf_counter()
    for nr in reps:
        tr = time.perf_counter()
        dt = advance(nr, dt)
        rep_rates.append(n1 * n2 * n3 * nr / (time.perf_counter() - tr))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    g.grmhd_profile(sim.ctx, False)
    kernels = {name: g.grmhd_profile_read(sim.ctx, name) for name in TIMED_KERNELS}
    # the remaining classes, every launch bracketed, outside the timed region
    others = [name for name in g.KERNELS if name not in TIMED_KERNELS]
    other_steps = min(args.steps, 5)
    g.grmhd_profile_kernels(sim.ctx, others)
    g.grmhd_profile(sim.ctx, True)
    dt = advance(other_steps, dt)
    g.grmhd_profile(sim.ctx, False)
    g.grmhd_profile_kernels(sim.ctx, list(g.KERNELS))
    kernels.update({name: g.grmhd_profile_read(sim.ctx, name) for name in others})
    fails = sim.step_failures()
    divb = sim.divb(P)
    zones = n1 * n2 * n3
    value = zones * args.steps / secs
    print("[bench] kernel ms/launch: " + ", ".join(
        f"{k} {ms / max(n, 1):.3f}" for k, (ms, n) in kernels.items()), file=sys.stderr, flush=True)

    # roofline of the dominant kernel (the fused update: CT, source, U(P),
    # inversion, bounds; one launch per substep = Z/2 zone-cycles) with the
    # method's compulsory bytes per zone-cycle as the algorithmic bytes
    dom = max(("sweeps", "update"), key=lambda k: kernels[k][0])
    ms, n = kernels[dom]
    t_launch = ms / n / 1e3
    per_zc = compulsory_bytes_per_zone_cycle(prm)
    per_launch = per_zc * zones / 2
    achieved = per_launch / t_launch
    workload = f"{'cks_bondi' if cks else 'fm_torus'}_{n1}x{n2}x{n3}_{args.recon}_{args.precision}"
    if args.electrons:
        workload += f"_electrons_{args.electrons}"
    traffic = measured_traffic(workload)
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK,
                "traffic": traffic[dom]["bytes_per_launch"] if traffic and dom in traffic else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "kernel": dom, "mean_launch_ms": ms / n,
                "algorithmic_bytes_per_launch": per_launch,
                "algorithmic_basis": (f"{per_zc:.2f} B per zone-cycle (P^n, P_h, P^n+1 traffic of the two substeps "
                                      + ("plus the 3D geometry tables of every zone" if cks else
                                         "plus the 2D geometry over n3")
                                      + f") x {zones} zones / 2 (one substep)")}
    if traffic:
        step_traffic = sum(rec["bytes_per_launch"] * rec["launches_per_step"] for rec in traffic.values())
        roofline["traffic_ratio"] = {
            "per_launch": roofline["traffic"] / per_launch if roofline["traffic"] else None,
            "per_step": step_traffic / (per_zc * zones),
            "step_traffic_bytes": step_traffic}
    else:
        roofline["traffic_ratio"] = None

    if args.copy_calibration_gib > 0:
        nel = int(args.copy_calibration_gib * 2 ** 30) // 8
        a = torch.ones(nel, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # other views: the whole step's compulsory bytes at the measured step
    # rate; this split design's own per-launch byte model (face fluxes
    # included); measured bytes over time; against the nominal peak and a
    # plain device copy measured here
    copy_bw = device_copy_bandwidth(torch, dev)
    split = split_design_bytes(dom, prm, mixed)
    views = {"copy_GBps": copy_bw / 1e9,
             "step_compulsory_bytes_per_zone_cycle": per_zc,
             "step_compulsory_frac": value * per_zc / HBM_PEAK,
             "step_compulsory_frac_of_copy": value * per_zc / copy_bw,
             "split_design_bytes_per_launch": split,
             "split_design_frac": split / t_launch / HBM_PEAK}
    if roofline["traffic"]:
        views["measured_frac"] = roofline["traffic"] / t_launch / HBM_PEAK
        views["measured_frac_of_copy"] = roofline["traffic"] / t_launch / copy_bw
    # the VALU view: counted FP64 / FP32 flops per launch over the live mean
    # launch time, against the vector peaks
    flops = measured_flops(workload)
    if flops:
        valu = {}
        for k, rec in flops.items():
            if k in kernels and kernels[k][1]:
                t = kernels[k][0] / kernels[k][1] / 1e3
                valu[k] = {"fp64_TFLOPs": rec["fp64"] / t / 1e12, "fp64_frac": rec["fp64"] / t / FP64_PEAK,
                           "fp32_TFLOPs": rec["fp32"] / t / 1e12, "fp32_frac": rec["fp32"] / t / FP32_PEAK}
        views["valu"] = valu
        if all(k in flops and kernels.get(k, (0, 0))[1] for k in ("sweeps", "update")):
            # FP64 work of a step: the two hot kernels' counted flops per launch
            # times their launches per step (the ghosts, fixup and dt are bytes)
            per_step = sum(flops[k]["fp64"] * kernels[k][1] / args.steps for k in ("sweeps", "update"))
            views["arithmetic_ceiling"] = arithmetic_ceiling(per_step, zones, per_zc, secs / args.steps)
    roofline["views"] = views

    if args.electrons:
        # the electron passes of a step (scalar ghosts, advection, heating, two
        # substeps each) against their own compulsory bytes: advection reads
        # rho and u~ of the base state, both entropies of the base and the flux
        # state and the three mass fluxes and writes U_K; heating reads the
        # new primitives and U_K and writes both entropies
        fb = 4 if mixed else 8
        per_zone = 2 * ((4 + 2 + 2 + 2) * 8 + 3 * fb + (8 + 2 + 2) * 8)
        # the electron classes are timed in the pass after the timed region
        e_ms = kernels["electrons"][0] / other_steps
        roofline["electron_passes"] = {"ms_per_step": e_ms, "algorithmic_bytes_per_zone_cycle": per_zone,
                                       "achieved_GBps": per_zone * zones / (e_ms / 1e3) / 1e9,
                                       "frac": per_zone * zones / (e_ms / 1e3) / HBM_PEAK}

    out = {
        "metric": "zone-cycles/s per GPU + % HBM roofline; batched-serving p50/p99 job latency",
        "value": value,
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not mixed else "f32+f64",
        "data": "synthetic",
        "config": {"workload": workload,
                   "grid": [n1, n2, n3], "a": prm["a"], "recon": args.recon,
                   "precision": args.precision, "coords": args.coords,
                   **({"box": [[prm["x1min"], prm["x1max"]], [prm["x2min"], prm["x2max"]],
                               [prm["x3min"], prm["x3max"]]]} if cks else {"r_out": 1000.0}),
                   "driver": args.path,
                   "electrons": args.electrons},
        "repeats": {"n": nrep, "steps": reps, "zone_cycles_per_s": rep_rates,
                    "median": sorted(rep_rates)[len(rep_rates) // 2]},
        "roofline": roofline,
        "kernels_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in kernels.items()},
        "checks": {"max_divb": divb, "failed_inversions_last_step": fails, "dt": dt},
    }
    sim.close()
    del P
    torch.cuda.empty_cache()
    if not args.no_many and not args.electrons and not cks:
        # the batched form against the per-job FP64 loop, a few steps of the
        # 64-job mix with tuned batch tiles
        out["many"] = many_record(args.many_steps, 1, True)
    if not args.no_serving and not args.electrons and not cks:
        print("[bench] serving stream", file=sys.stderr, flush=True)
        out["serving"] = serving_record()
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_cks(prm) if cks else cpu_baseline(prm)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
