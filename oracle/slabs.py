"""The oracle's predictor-corrector step on a large grid, by x3 slabs in
parallel worker processes (test infrastructure only, like the rest of
``oracle``).

Nothing here changes what is computed: each substep of ``oracle.step`` is
evaluated on windows of x3 planes by ``oracle.step.substep`` itself, and the
windows are wide enough that every plane a worker keeps equals the
whole-domain substep bit for bit (pinned by ``tests/test_oracle_step.py``):

* a worker that owns interior planes k0..k1-1 runs the substep on planes
  k0-1..k1 (one extra plane per side, so that the fixup of a kept plane sees
  its neighbours' failure flags and values), with NG = 3 neighbour planes per
  side as the window's x3 ghosts (the reconstruction stencil and Flux-CT need
  no more), and keeps k0..k1-1;
* between substeps the parent fills the ghost zones of the whole domain
  (``oracle.step.fill_ghosts``), exactly as ``oracle.step.step`` does;
* the Courant step takes the maximum of the workers' corrector signal speeds.

The x3 direction must be periodic (the benchmark torus); memory per worker is
about 1-2 GB for a 288 x 128 grid with 8-plane slabs.
"""

import multiprocessing as mp
import os
import sys
import time
from multiprocessing import shared_memory

import numpy as np

from .grid import Grid, NG
from .step import fill_ghosts, substep, dt_from_ctop, BC_PERIODIC

_W = {}          # per worker: the grid and the attached shared arrays


def _attach(names, shape):
    arrs, shms = {}, []
    for key, name in names.items():
        shm = shared_memory.SharedMemory(name=name)
        shms.append(shm)
        arrs[key] = np.ndarray(shape, dtype=np.float64, buffer=shm.buf)
    return arrs, shms


def _init_worker(prm, names, shape):
    arrs, shms = _attach(names, shape)
    _W["grid"] = Grid(prm)
    _W["a"] = arrs
    _W["shm"] = shms


def _window(A, k_lo, k_hi, n3):
    """Planes k_lo..k_hi-1 (interior numbering, wrapped periodically) of padded A."""
    ks = np.arange(k_lo, k_hi) % n3 + NG
    return A[:, ks]


def _work(task):
    """One substep on a slab: task = (src, base, dst, k0, k1, dt), the names of
    the shared arrays holding the flux state (ghosts filled), the base state and
    the output. Returns the slab's failure count and per-direction
    signal-speed maxima."""
    src, base_key, dst, k0, k1, dt = task
    grid = _W["grid"]
    a = _W["a"]
    n1, n2, n3 = grid.n
    blk = _window(a[src], k0 - 1 - NG, k1 + 1 + NG, n3)
    base = _window(a[base_key], k0 - 1, k1 + 1, n3)[:, :, NG:NG + n2, NG:NG + n1]
    Pi, failed, cmax = substep(blk, base, grid, dt, window=True)
    a[dst][:, NG + k0:NG + k1, NG:NG + n2, NG:NG + n1] = Pi[:, 1:-1]
    return int(failed[1:-1].sum()), cmax


def _speeds(task):
    """Per-direction maximum signal speeds of a state on a slab, the faces that
    oracle.get_dt takes (task = (name of the state, k0, k1))."""
    from .step import face_fluxes
    key, k0, k1 = task
    grid = _W["grid"]
    n1, n2, n3 = grid.n
    blk = _window(_W["a"][key], k0 - NG, k1 + NG, n3)
    K, J, I = slice(NG, NG + k1 - k0), slice(NG, NG + n2), slice(NG, NG + n1)
    C1 = face_fluxes(blk, grid, 1)[1]
    C2 = face_fluxes(blk, grid, 2)[1]
    C3 = face_fluxes(blk, grid, 3)[1]
    return (np.nanmax(C1[K, J, NG:NG + n1 + 1]), np.nanmax(C2[K, NG:NG + n2 + 1, I]),
            np.nanmax(C3[NG:NG + (k1 - k0) + 1, J, I]))


def _slabs(n3, width):
    return [(k, min(k + width, n3)) for k in range(0, n3, width)]


def run(prm, P0, nsteps, dts=None, workers=None, width=None, log=None):
    """Evolve the padded state P0 by nsteps oracle steps.

    dts: the step sizes to use (list of nsteps), or None for the oracle's own
    sequence dt_0 = get_dt(P0), dt_{n+1} = min(dt_next, 1.3 dt_n) (as
    ``oracle.run``). Returns (P, dts used, failed inversions per step).
    workers: processes (default min(16, cpu count)); width: planes per slab.
    log: a callable taking a progress string (one line per substep).
    """
    n3 = prm["n3"]
    if list(prm["bc"][2]) != [BC_PERIODIC, BC_PERIODIC]:
        raise ValueError("the slab driver needs a periodic x3 direction")
    workers = workers or min(16, os.cpu_count() or 1)
    width = width or max(1, -(-n3 // workers))
    shape = P0.shape
    nbytes = int(np.prod(shape)) * 8
    shms = {k: shared_memory.SharedMemory(create=True, size=nbytes) for k in ("A", "B", "C")}
    try:
        arrs = {k: np.ndarray(shape, dtype=np.float64, buffer=s.buf) for k, s in shms.items()}
        cur, half, nxt = "A", "B", "C"
        arrs[cur][:] = P0
        grid = Grid(prm)
        names = {k: s.name for k, s in shms.items()}
        slabs = _slabs(n3, width)
        used, fails = [], []
        dt = None if dts is None else dts[0]
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(workers, initializer=_init_worker, initargs=(prm, names, shape)) as pool:
            for step in range(nsteps):
                fill_ghosts(arrs[cur], grid)
                if dt is None:
                    out = pool.map(_speeds, [(cur, k0, k1) for k0, k1 in slabs])
                    dt = dt_from_ctop(tuple(max(o[d] for o in out) for d in range(3)), grid)
                used.append(dt)
                # ghost zones of P_h start as P^n's (Dirichlet ghosts are kept by the fill)
                arrs[half][:] = arrs[cur]
                res = pool.map(_work, [(cur, cur, half, k0, k1, 0.5 * dt) for k0, k1 in slabs])
                nf = sum(r[0] for r in res)
                fill_ghosts(arrs[half], grid)
                if log:
                    log(f"oracle step {step}: predictor done ({time.perf_counter() - t0:.1f} s)")
                arrs[nxt][:] = arrs[cur]
                res = pool.map(_work, [(half, cur, nxt, k0, k1, dt) for k0, k1 in slabs])
                nf += sum(r[0] for r in res)
                fails.append(nf)
                cmax = tuple(max(r[1][d] for r in res) for d in range(3))
                cur, nxt = nxt, cur
                if log:
                    log(f"oracle step {step}: corrector done, {nf} failed inversions "
                        f"({time.perf_counter() - t0:.1f} s)")
                if dts is not None:
                    dt = dts[step + 1] if step + 1 < len(dts) else None
                else:
                    dt = min(dt_from_ctop(cmax, grid), 1.3 * dt)
        return arrs[cur].copy(), used, fails
    finally:
        for s in shms.values():
            s.close()
            s.unlink()


def stderr_log(msg):
    print(msg, file=sys.stderr, flush=True)
