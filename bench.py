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
steps (bracketed by device synchronisation). Kernel durations over the same
timed region come from HIP events the library records on its stream around
every launch; the dominant kernel's algorithmic bytes per launch over its mean
duration give the roofline fraction against 8 TB/s. The oracle (NumPy FP64,
one core) is timed on a bounded sample of the same workload.

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


def algorithmic_bytes(kernel, prm, mixed):
    """Bytes one launch must move at minimum: every input value read once and
    every output written once (stencil re-reads are cache traffic, not algorithm).
    """
    n1, n2, n3 = prm["n1"], prm["n2"], prm["n3"]
    fb = 4 if mixed else 8
    recon_reach = 3 if prm["recon"] == 1 else 2          # zones below / above+1 a face
    if kernel in ("sweep1", "sweep2", "sweep3"):
        d = int(kernel[-1])
        n = [n1, n2, n3]
        faces = 1
        cells = 1
        for e in range(3):
            if e == d - 1:
                faces *= n[e] + 1
                cells *= n[e] + 2 * recon_reach
            else:
                faces *= n[e] + 2
                cells *= n[e] + 2
        geo = 22 * fb * (n1 + 2) * (n2 + 2)
        return 64 * cells + 8 * fb * faces + geo
    if kernel == "update":
        zones = n1 * n2 * n3
        # 7 flux components per direction (5 hydro + 2 transverse B); the states
        # read: one in the predictor (P_base = P_s = P), two in the corrector
        # (P, P_h), 96 B a zone on average over the two launches of a step;
        # P_out written; one flag byte; the 2D centre table once
        return zones * (21 * fb + 96 + 64 + 1) + 64 * 8 * n1 * n2
    raise KeyError(kernel)


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


def measured_traffic(kernel, workload):
    """HBM bytes per launch of ``kernel`` from the committed counter summary
    (profiles/hbm_traffic.json: FETCH_SIZE and WRITE_SIZE scaled by a plain
    copy), only while the library is the build those counters were taken on."""
    path = os.path.join(HERE, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        from paper_2110_10191_amd import tune
        if (rec.get("kernel") == kernel and rec.get("workload") == workload
                and rec.get("library_hash") == tune.library_hash()):
            return float(rec["bytes_per_launch"])
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
    return {
        "value": zones * nsteps / secs,
        "unit": "zone-cycles/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{nsteps} FP64 steps of the {prm['n1']}x{prm['n2']} FMKS torus grid with {nslabs} x3 slabs "
                   f"({zones} zones, same per-zone work as the benchmark grid) in {secs:.1f} s; "
                   "NumPy element-wise, single thread"),
    }


def bench_many(args):
    """64 independent uneven jobs (32 periodic boxes N^3, N in 32..96; 32 Bondi
    flows in Kerr, a ~ U[0, 0.99], up to 192 x 128 x 64): every job advanced
    by the batch calls (one grid per kernel phase over all jobs, a captured
    HIP graph per step, per-job dt on the device), in FP64 and in mixed
    precision, against the plain loop that steps one job after another in
    FP64 with a host-side dt per step."""
    import torch
    import paper_2110_10191_amd as g
    from paper_2110_10191_amd import tune
    import problems
    from problems.workloads import many_jobs

    specs = many_jobs(64, seed=3)
    zones = sum(s.zones for s in specs)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    res = {}
    for prec_name, prec in (("fp64", problems.FP64), ("mixed", problems.MIXED)):
        t_gen = time.perf_counter()
        sims, states = [], []
        for sp in specs:
            prm, P0 = sp.make(recon=problems.RECON_MC, precision=prec)
            sim = g.Sim(prm, device=dev)
            sims.append(sim)
            states.append(sim.to_device(P0))
        torch.cuda.synchronize()
        print(f"[bench] {prec_name}: {len(specs)} jobs, {zones} zones set up in "
              f"{time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
        tiles = None
        if args.tune:
            tiles, _ = tune.tune_batch(sims, states, steps=2, repeats=1)
            print(f"[bench] {prec_name}: batch tiles {tiles}", file=sys.stderr, flush=True)
        dts = [s.get_dt(P) for s, P in zip(sims, states)]
        b = g.Batch(sims)
        b.set_dt(dts)
        b.step(states, nsteps=args.warmup)
        b.get()
        t0 = time.perf_counter()
        b.step(states, nsteps=args.steps)
        _, status = b.get()
        secs = time.perf_counter() - t0
        b.close()
        res[f"batched_{prec_name}"] = {"value": zones * args.steps / secs, "ms_per_step": secs / args.steps * 1e3,
                                       "tiles": tiles, "bad_jobs": int(sum(status))}
        print(f"[bench] batched {prec_name}: {zones * args.steps / secs:.3e} zone-cycles/s",
              file=sys.stderr, flush=True)
        if prec == problems.FP64:
            dts = [s.get_dt(P) for s, P in zip(sims, states)]
            for s, P, dt in zip(sims, states, dts):
                s.step(P, dt)                        # warm each job's code path
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for s, P, dt in zip(sims, states, dts):
                for _ in range(args.steps):
                    dt = min(s.step(P, dt), 1.3 * dt)
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            res["per_job_loop_fp64"] = {"value": zones * args.steps / secs,
                                        "ms_per_step": secs / args.steps * 1e3}
            print(f"[bench] per-job FP64 loop: {zones * args.steps / secs:.3e} zone-cycles/s",
                  file=sys.stderr, flush=True)
        for s in sims:
            s.close()
        del states
        torch.cuda.empty_cache()
    base = res["per_job_loop_fp64"]["value"]
    out = {
        "metric": "zone-cycles/s, batched uneven jobs vs the per-job FP64 loop",
        "value": res["batched_mixed"]["value"],
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["batched_mixed"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "64 uneven jobs: 32 boxes N^3 (N in 32..96), 32 Kerr Bondi (up to 192x128x64), MC",
                   "zones": zones, "seed": 3},
        "batched_fp64": res["batched_fp64"],
        "batched_mixed": res["batched_mixed"],
        "per_job_loop_fp64": res["per_job_loop_fp64"],
        "speedup_batched_mixed_vs_loop": res["batched_mixed"]["value"] / base,
        "speedup_batched_fp64_vs_loop": res["batched_fp64"]["value"] / base,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--recon", choices=["mc", "weno5"], default="mc")
    ap.add_argument("--grid", type=int, nargs=3, default=[288, 128, 128])
    ap.add_argument("--no-cpu-baseline", action="store_true")
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
    n1, n2, n3 = args.grid
    t_gen = time.perf_counter()
    prm, P0 = problems.fm_torus(n1=n1, n2=n2, n3=n3, recon=recon,
                                precision=problems.MIXED if mixed else problems.FP64)
    print(f"[bench] initial data {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sim = g.Sim(prm, device=dev)
    P = sim.to_device(P0)
    torch.cuda.synchronize()

    dt = sim.get_dt(P)
    kernels = {}
    if args.electrons and args.path == "device":
        # the fluid step plus the three electron passes per substep, through
        # grmhd_run_electrons (the step size kept on the device)
        E = sim.to_device(problems.electron_scalars(P0, prm["gam"]))
        dt = sim.run_electrons(P, E, args.warmup, dt, args.electrons)
        print(f"[bench] warmup done, dt = {dt:.3e}", file=sys.stderr, flush=True)
        g.grmhd_profile(sim.ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dt = sim.run_electrons(P, E, args.steps, dt, args.electrons)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        g.grmhd_profile(sim.ctx, False)
        for name in g.KERNELS:
            kernels[name] = g.grmhd_profile_read(sim.ctx, name)
    elif args.electrons:
        # one grmhd_step_electrons call per step, dt read back every step
        E = sim.to_device(problems.electron_scalars(P0, prm["gam"]))
        for _ in range(args.warmup):
            dt = min(sim.step_electrons(P, E, dt, args.electrons), 1.3 * dt)
        torch.cuda.synchronize()
        print(f"[bench] warmup done, dt = {dt:.3e}", file=sys.stderr, flush=True)
        g.grmhd_profile(sim.ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dt = min(sim.step_electrons(P, E, dt, args.electrons), 1.3 * dt)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        g.grmhd_profile(sim.ctx, False)
        for name in g.KERNELS:
            kernels[name] = g.grmhd_profile_read(sim.ctx, name)
    elif args.path == "host":
        # one grmhd_step call per step; dt read back to the host every step
        for _ in range(args.warmup):
            dt = min(sim.step(P, dt), 1.3 * dt)
        torch.cuda.synchronize()
        print(f"[bench] warmup done, dt = {dt:.3e}", file=sys.stderr, flush=True)
        g.grmhd_profile(sim.ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            dt = min(sim.step(P, dt), 1.3 * dt)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        g.grmhd_profile(sim.ctx, False)
        for name in g.KERNELS:
            kernels[name] = g.grmhd_profile_read(sim.ctx, name)
    else:
        # grmhd_run: the same kernels with the step size kept on the device
        # (dt <- min(dt_next, 1.3 dt) by a one-thread kernel), so the host
        # never waits between steps; every launch is bracketed by events
        dt = sim.run(P, args.warmup, dt)
        print(f"[bench] warmup done, dt = {dt:.3e}", file=sys.stderr, flush=True)
        g.grmhd_profile(sim.ctx, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dt = sim.run(P, args.steps, dt)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        g.grmhd_profile(sim.ctx, False)
        for name in g.KERNELS:
            kernels[name] = g.grmhd_profile_read(sim.ctx, name)
    fails = sim.step_failures()
    divb = sim.divb(P)
    zones = n1 * n2 * n3
    value = zones * args.steps / secs
    print("[bench] kernel ms/launch: " + ", ".join(
        f"{k} {ms / max(n, 1):.3f}" for k, (ms, n) in kernels.items()), file=sys.stderr, flush=True)

    dom = max(("sweep1", "sweep2", "sweep3", "update"), key=lambda k: kernels[k][0])
    ms, n = kernels[dom]
    per_launch = algorithmic_bytes(dom, prm, mixed)
    achieved = per_launch / (ms / n / 1e3)
    workload = f"fm_torus_{n1}x{n2}x{n3}_{args.recon}_{args.precision}"
    if args.electrons:
        workload += f"_electrons_{args.electrons}"
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achieved / HBM_PEAK, "traffic": measured_traffic(dom, workload),
                "traffic_unit": "bytes per launch", "kernel": dom,
                "algorithmic_bytes_per_launch": per_launch, "mean_launch_ms": ms / n}

    if args.copy_calibration_gib > 0:
        nel = int(args.copy_calibration_gib * 2 ** 30) // 8
        a = torch.ones(nel, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # the other two views of the HBM roofline: the whole step's compulsory
    # state traffic (read P^n, write P_h; read P^n and P_h, write P^{n+1}:
    # 320 B a zone, plus the 2D geometry once per step) at the measured rate,
    # and the dominant kernel's measured HBM bytes over its time; both against
    # the nominal peak and against a plain device copy measured here
    copy_bw = device_copy_bandwidth(torch, dev)
    step_bytes = 320.0 * zones + 2 * 150 * 8 * n1 * n2
    views = {"copy_GBps": copy_bw / 1e9,
             "step_compulsory_bytes_per_zone_cycle": step_bytes / zones,
             "step_compulsory_frac": value * step_bytes / zones / HBM_PEAK,
             "step_compulsory_frac_of_copy": value * step_bytes / zones / copy_bw}
    if roofline["traffic"]:
        views["measured_frac"] = roofline["traffic"] / (ms / n / 1e3) / HBM_PEAK
        views["measured_frac_of_copy"] = roofline["traffic"] / (ms / n / 1e3) / copy_bw
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
    roofline["views"] = views

    if args.electrons:
        # the electron passes of a step (scalar ghosts, advection, heating, two
        # substeps each) against their own compulsory bytes: advection reads
        # rho and u~ of the base state, both entropies of the base and the flux
        # state and the three mass fluxes and writes U_K; heating reads the
        # new primitives and U_K and writes both entropies
        fb = 4 if mixed else 8
        per_zone = 2 * ((4 + 2 + 2 + 2) * 8 + 3 * fb + (8 + 2 + 2) * 8)
        e_ms = kernels["electrons"][0] / args.steps
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
                   "precision": args.precision, "coords": "fmks", "r_out": 1000.0,
                   "driver": args.path,
                   "electrons": args.electrons},
        "roofline": roofline,
        "kernels_ms_per_launch": {k: v[0] / max(v[1], 1) for k, v in kernels.items()},
        "checks": {"max_divb": divb, "failed_inversions_last_step": fails, "dt": dt},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(prm)
    sim.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
