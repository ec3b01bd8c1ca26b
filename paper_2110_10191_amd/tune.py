"""Tile autotuner for the stencil kernels.

The sweep kernels (face fluxes) and the update/fixup kernels each take a
thread-block tile of tx zones along x1 by ty rows along x2 (one thread per
zone; a launch covers x3 in XCD-contiguous chunks). The best tile depends on
the grid's x1 extent (a tile wider than n1 idles lanes), on the reconstruction
(stencil reach) and on the precision (register pressure), so the tuner times
each candidate on the device and keeps the fastest per

    (device, library build, reconstruction, precision, grid bucket)

in a JSON cache. Sweep and update tiles are independent launch parameters of
different kernels, so each class is tuned with the other held fixed. The
objective is the median over repeats of the summed kernel time of that class
per step, read from the HIP events the library brackets its launches with.

Tiles never change results (each zone or face is one thread's work from the
same operands, and the only reductions are maxima and counts), so a tuned tile
is safe to apply to any problem in its bucket.

    from paper_2110_10191_amd import tune
    tiles = tune.tune_problem(prm, P0)           # time, cache, return
    tune.apply(sim)                               # set cached tiles, if any
"""

import hashlib
import json
import os
import statistics

from . import _binding as B

# x1 tile widths and rows per block; waves per block = tx * ty / 64
WIDTHS = (32, 64, 128, 256)
ROWS = (1, 2, 4, 8, 16)
MAX_THREADS = {"sweep": 512, "update": 256}   # the kernels' launch bounds
DEFAULT = {"sweep": (64, 8), "update": (64, 1)}

SWEEP_CLASSES = ("sweeps",)
UPDATE_CLASSES = ("update", "fixup")

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "grmhd", "tiles.json")


def candidates(cls="update"):
    """Every legal tile of the candidate set for a kernel class: tx * ty a
    multiple of 64, at most the class's launch bound."""
    out = []
    for tx in WIDTHS:
        for ty in ROWS:
            n = tx * ty
            if n % 64 == 0 and n <= MAX_THREADS[cls]:
                out.append((tx, ty))
    return out


def _bucket_n(n):
    """Smallest power of two >= n (at least 8)."""
    b = 8
    while b < n:
        b *= 2
    return b


def bucket(prm):
    """Grid bucket of a problem: x1 extent and zone count, each rounded up to
    a power of two, plus reconstruction and precision."""
    zones = prm["n1"] * prm["n2"] * prm["n3"]
    recon = "weno5" if prm["recon"] == 1 else "mc"
    prec = "mixed" if prm["precision"] == 1 else "fp64"
    return f"{recon}/{prec}/n1<={_bucket_n(prm['n1'])}/zones<={_bucket_n(zones)}"


def library_hash(path=None):
    """Short content hash of the built library: tuned tiles are only valid for
    the kernels they were timed on."""
    h = hashlib.sha256()
    with open(path or B.LIB_PATH, "rb") as f:
        for chunk in iter(lambda: f.read(1 << 20), b""):
            h.update(chunk)
    return h.hexdigest()[:16]


def device_key():
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "")
    return f"{props.name}|{arch}|cu{props.multi_processor_count}"


class TileCache:
    """JSON file {device|library: {bucket: {"sweep": [tx, ty], "update": [tx, ty], ...}}}."""

    def __init__(self, path=None, device=None, lib_hash=None):
        self.path = path or os.environ.get("GRMHD_TILE_CACHE", DEFAULT_CACHE)
        self._device = device
        self._lib = lib_hash

    @property
    def scope(self):
        if self._device is None:
            self._device = device_key()
        if self._lib is None:
            self._lib = library_hash()
        return f"{self._device}|{self._lib}"

    def load(self):
        try:
            with open(self.path) as f:
                data = json.load(f)
        except (OSError, ValueError):
            return {}
        return data if isinstance(data, dict) else {}

    def get(self, key):
        entry = self.load().get(self.scope, {}).get(key)
        if not entry:
            return None
        tiles = {}
        for cls in ("sweep", "update"):
            t = entry.get(cls)
            if t is None or tuple(t) not in candidates(cls):
                return None
            tiles[cls] = tuple(t)
        return tiles

    def put(self, key, tiles, timings=None):
        data = self.load()
        entry = {cls: list(tiles[cls]) for cls in ("sweep", "update")}
        if timings:
            entry["ms_per_step"] = timings
        data.setdefault(self.scope, {})[key] = entry
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = f"{self.path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def pick(times):
    """Fastest candidate of {tile: [per-repeat ms]} by median; ties keep the
    earlier candidate (the candidate order puts the default first)."""
    best, best_t = None, None
    for tile, ts in times.items():
        m = statistics.median(ts)
        if best_t is None or m < best_t:
            best, best_t = tile, m
    return best, best_t


def _ordered(cls, default=None):
    default = default or DEFAULT[cls]
    return [default] + [t for t in candidates(cls) if t != default]


def time_classes(sim, P, dt, classes, steps, repeats):
    """Per-repeat summed kernel ms per step of the given classes."""
    out = []
    for _ in range(repeats):
        B.grmhd_profile(sim.ctx, True)
        for _ in range(steps):
            sim.step(P, dt, want_dt_next=False)
        total = 0.0
        for k in classes:
            ms, _ = B.grmhd_profile_read(sim.ctx, k)
            total += ms
        B.grmhd_profile(sim.ctx, False)
        out.append(total / steps)
    return out


def tune_sim(sim, P, steps=3, repeats=3):
    """Time every candidate tile for the sweep and the update classes, each
    starting from state P (restored afterwards), and return
    ({"sweep": t, "update": t}, {"sweep": ms, "update": ms}). Leaves the best
    tiles set on ``sim``. Every candidate runs one untimed step first, and the
    repeats go round all candidates in turn, so neither warm-up nor drift of
    the device favours the candidates timed first."""
    P0 = P.clone()
    dt = sim.get_dt(P)
    result, timings = {}, {}
    for cls, classes in (("sweep", SWEEP_CLASSES), ("update", UPDATE_CLASSES)):
        order = _ordered(cls)
        times = {tile: [] for tile in order}
        for tile in order:
            sim.set_tiles(cls, *tile)
            P.copy_(P0)
            sim.step(P, dt, want_dt_next=False)
        for _ in range(repeats):
            for tile in order:
                sim.set_tiles(cls, *tile)
                P.copy_(P0)
                times[tile] += time_classes(sim, P, dt, classes, steps, 1)
        best, best_ms = pick(times)
        sim.set_tiles(cls, *best)
        result[cls] = best
        timings[cls] = best_ms
        timings[cls + "_all"] = {f"{tx}x{ty}": statistics.median(ts) for (tx, ty), ts in times.items()}
    P.copy_(P0)
    return result, timings


def search(measure, repeats=3):
    """Coordinate search over the two tile classes with a caller's timer.

    measure(tiles) -> seconds (or ms) of some fixed work run with
    tiles = {"sweep": (tx, ty), "update": (tx, ty)}. The sweep tile is chosen
    with the update tile at its default, then the update tile with the chosen
    sweep tile. Returns (tiles, {cls: best median})."""
    tiles = dict(DEFAULT)
    best_t = {}
    for cls in ("sweep", "update"):
        order = _ordered(cls)
        times = {tile: [] for tile in order}
        # the repeats go round all candidates in turn (no drift favours the first)
        for _ in range(repeats):
            for tile in order:
                times[tile].append(measure(dict(tiles, **{cls: tile})))
        tiles[cls], best_t[cls] = pick(times)
    return tiles, best_t


def tune_batch(sims, states, steps=3, repeats=3, stream=None):
    """Tiles for a batch of Sim objects (the batch takes its first job's tiles),
    timed on whole batched steps; the states advance. Leaves the best tiles set
    on sims[0] and returns them with their per-step times in ms."""
    import time
    import torch

    dts = [s.get_dt(P) for s, P in zip(sims, states)]

    def measure(tiles):
        sims[0].set_tiles("sweep", *tiles["sweep"])
        sims[0].set_tiles("update", *tiles["update"])
        b = B.Batch(sims, stream=stream)
        try:
            b.set_dt(dts)
            b.step(states, nsteps=1)             # capture + warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            b.step(states, nsteps=steps)
            b.get()                              # synchronises the batch stream
            return (time.perf_counter() - t0) / steps * 1e3
        finally:
            b.close()

    tiles, best = search(measure, repeats=repeats)
    sims[0].set_tiles("sweep", *tiles["sweep"])
    sims[0].set_tiles("update", *tiles["update"])
    return tiles, best


def tune_problem(prm, P0, cache=None, force=False, steps=3, repeats=3, device="cuda:0"):
    """Tiles for problem ``prm`` (initial state P0, host array in the generator
    layout): from the cache when present, else timed on a scratch copy and
    stored."""
    cache = cache or TileCache()
    key = bucket(prm)
    if not force:
        hit = cache.get(key)
        if hit:
            return hit
    sim = B.Sim(prm, device=device)
    try:
        P = sim.to_device(P0)
        tiles, timings = tune_sim(sim, P, steps=steps, repeats=repeats)
    finally:
        sim.close()
    cache.put(key, tiles, timings)
    return tiles


def apply(sim, cache=None):
    """Set the cached tiles for ``sim``'s bucket; returns them, or None (the
    library default stays) when the bucket was never tuned."""
    cache = cache or TileCache()
    tiles = cache.get(bucket(sim.prm))
    if tiles:
        sim.set_tiles("sweep", *tiles["sweep"])
        sim.set_tiles("update", *tiles["update"])
    return tiles
