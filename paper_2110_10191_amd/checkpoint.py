"""Checkpoint and restart of a run.

A checkpoint holds everything the step needs to continue bit for bit: the
primitive state with its ghost zones (the generator layout
[8, n3+6, n2+6, n1+6], float64), the problem (the fields of
``grmhd_problem``), the step size for the next step, the time and the step
count. Geometry is not stored: a context rebuilds it deterministically from
the problem. The file is a NumPy ``.npz`` archive of plain arrays and a JSON
string, read back without unpickling anything. A run with electron heating
also stores its two entropies ([2, n3+6, n2+6, n1+6], float64) and its
heating model and constant fraction.

    from paper_2110_10191_amd import checkpoint
    checkpoint.save(path, sim.prm, sim.to_host(P), dt, t, step)
    ck = checkpoint.load(path)
    sim = Sim(ck.prm); P = sim.to_device(ck.P); dt = ck.dt
    # with electron heating: save(..., E=sim.to_host(E), heat=("howes", 0.0)),
    # then E = sim.to_device(ck.E) and ck.heat
"""

import json
import os
from dataclasses import dataclass

import numpy as np

FORMAT = 1


@dataclass
class Checkpoint:
    prm: dict
    P: np.ndarray
    dt: float
    t: float
    step: int
    E: np.ndarray = None      # electron entropies, or None
    heat: tuple = None        # (model, fel) of the electron heating, or None


def _problem_json(prm):
    # only JSON-representable fields; bookkeeping keys starting with "_" that
    # are not (large arrays, objects) are dropped
    out = {}
    for k, v in prm.items():
        try:
            json.dumps(v)
        except TypeError:
            continue
        out[k] = v
    return json.dumps(out, sort_keys=True)


def save(path, prm, P, dt, t=0.0, step=0, E=None, heat=None):
    """Write a checkpoint atomically (temporary file, then rename). E and heat
    = (model, fel): the electron entropies and heating of a run that has them."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    shape = (8, prm["n3"] + 6, prm["n2"] + 6, prm["n1"] + 6)
    if P.shape != shape:
        raise ValueError(f"state shape {P.shape} is not {shape}")
    if not (dt > 0.0 and np.isfinite(dt)):
        raise ValueError("dt must be finite and > 0")
    extra = {}
    if E is not None:
        E = np.ascontiguousarray(E, dtype=np.float64)
        if E.shape != (2,) + shape[1:]:
            raise ValueError(f"entropy shape {E.shape} is not {(2,) + shape[1:]}")
        if heat is None:
            raise ValueError("entropies need their heating (model, fel)")
        extra = dict(E=E, heat=np.array(json.dumps([heat[0], float(heat[1])])))
    tmp = f"{path}.{os.getpid()}.tmp.npz"
    np.savez(tmp, format=np.int64(FORMAT), problem=np.array(_problem_json(prm)), P=P,
             dt=np.float64(dt), t=np.float64(t), step=np.int64(step), **extra)
    os.replace(tmp, path)


def load(path):
    with np.load(path, allow_pickle=False) as z:
        fmt = int(z["format"])
        if fmt != FORMAT:
            raise ValueError(f"checkpoint format {fmt}, expected {FORMAT}")
        prm = json.loads(str(z["problem"]))
        P = np.array(z["P"], dtype=np.float64)
        E = heat = None
        if "E" in z.files:
            E = np.array(z["E"], dtype=np.float64)
            model, fel = json.loads(str(z["heat"]))
            heat = (model, fel)
        return Checkpoint(prm=prm, P=P, dt=float(z["dt"]), t=float(z["t"]), step=int(z["step"]), E=E, heat=heat)
