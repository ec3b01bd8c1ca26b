"""Linear MHD eigenmodes on a periodic Minkowski box.

The linear-mode convergence problem of the Tests section: a uniform background
(rho = 1, u = 1, u~ = 0, B = (1, 0, 0), gamma = 4/3) on X in [0,1)^3 carrying
small-amplitude eigenmodes with wave vector k = 2 pi (kx, ky, kz). Each mode m
with right eigenvector R_m (in primitive variables) and frequency omega_m is
laid down as

  dP(x, t) = amp * Re[R_m exp(i (k.x - omega_m t + phi_m))],

with seeded phases phi_m = 2 pi U[0,1). The eigenvectors are stored in
``linear_modes.json`` beside this file (written by ``make_linear_modes.py``,
which solves the linearised problem with the CPU oracle).
"""

import json
import math
import os

import numpy as np

from .params import RECON_MC, FP64, base_problem, NG

_HERE = os.path.dirname(os.path.abspath(__file__))
MODES_FILE = os.path.join(_HERE, "linear_modes.json")

BACKGROUND = np.array([1.0, 1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0])
GAMMA = 4.0 / 3.0


def kkey(kvec):
    return ",".join(str(int(k)) for k in kvec)


def load_modes():
    with open(MODES_FILE) as f:
        return json.load(f)


def mode_solution(prm, t, ghosts=False):
    """Analytic primitives [8, n3, n2, n1] at time t (zone-centre point values)."""
    meta = prm["_modes"]
    n1, n2, n3 = prm["n1"], prm["n2"], prm["n3"]
    ext = NG if ghosts else 0
    x = (np.arange(-ext, n1 + ext) + 0.5) / n1
    y = (np.arange(-ext, n2 + ext) + 0.5) / n2
    z = (np.arange(-ext, n3 + ext) + 0.5) / n3
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    kx, ky, kz = (2.0 * math.pi * k for k in meta["kvec"])
    P = np.empty((8,) + X.shape)
    P[:] = BACKGROUND[:, None, None, None]
    for m in meta["modes"]:
        R = np.array(m["R_re"]) + 1j * np.array(m["R_im"])
        ph = kx * X + ky * Y + kz * Z - m["omega"] * t + m["phase"]
        P += meta["amp"] * np.real(R[:, None, None, None] * np.exp(1j * ph))
    return P


def linear_modes(n=32, seed=1, amp=1e-4, kvec=(1, 1, 1), modes=("slow", "alfven"),
                 recon=RECON_MC, precision=FP64, n3=None):
    n3 = n if n3 is None else n3
    table = load_modes()[kkey(kvec)]
    rng = np.random.default_rng(seed)
    phases = 2.0 * math.pi * rng.random(len(modes))
    meta = dict(kvec=list(kvec), amp=amp, modes=[
        dict(name=name, omega=table[name]["omega"], R_re=table[name]["R_re"],
             R_im=table[name]["R_im"], phase=float(ph)) for name, ph in zip(modes, phases)])
    prm = base_problem(n, n, n3, gam=GAMMA, recon=recon, precision=precision,
                       _name="linear_modes", _seed=seed, _modes=meta)
    P = np.zeros((8, n3 + 2 * NG, n + 2 * NG, n + 2 * NG))
    P[:, NG:NG + n3, NG:NG + n, NG:NG + n] = mode_solution(prm, 0.0)
    return prm, P
