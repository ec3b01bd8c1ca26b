"""Seeded job lists for the many-problem workloads.

Two synthetic mixes of independent problems of uneven size, drawn from the
problems the method evolves (Tests and Scaling sections: linear modes on a
box, Bondi accretion, the magnetised torus in Kerr):

* ``many_jobs`` -- a fixed list advanced together: jobs 0..31 are periodic
  boxes of N^3 zones, N in {32, 48, 64, 80, 96}; jobs 32..63 are Bondi flows
  with spin a ~ U[0, 0.99], N1 in {64, 96, ..., 192}, N2 in {64, 96, 128},
  N3 in {32, 48, 64};
* ``poisson_stream`` -- arrivals at Poisson rate lam: each job is a torus or a
  Bondi flow (probability 1/2 each), spin a ~ U[0, 0.99], the Bondi grid set
  above, and a step count ~ U{200, ..., 2000}.

A ``JobSpec`` only names the job; ``make`` places its initial data.
"""

from dataclasses import dataclass

import numpy as np

from .params import RECON_MC, FP64
from .modes import linear_modes
from .bondi import bondi
from .torus import fm_torus

BOX_N = (32, 48, 64, 80, 96)
KERR_N1 = tuple(range(64, 193, 32))
KERR_N2 = (64, 96, 128)
KERR_N3 = (32, 48, 64)


@dataclass(frozen=True)
class JobSpec:
    id: int
    kind: str                 # "box", "bondi" or "torus"
    n1: int
    n2: int
    n3: int
    a: float = 0.0
    steps: int = 0
    arrival: float = 0.0      # seconds after the stream starts

    @property
    def zones(self):
        return self.n1 * self.n2 * self.n3

    def make(self, recon=RECON_MC, precision=FP64):
        """(prm, P) of this job with the given reconstruction and precision."""
        if self.kind == "box":
            return linear_modes(n=self.n1, n3=self.n3, recon=recon, precision=precision)
        if self.kind == "bondi":
            return bondi(n1=self.n1, n2=self.n2, n3=self.n3, a=self.a, recon=recon, precision=precision)
        if self.kind == "torus":
            return fm_torus(n1=self.n1, n2=self.n2, n3=self.n3, a=self.a, recon=recon, precision=precision)
        raise ValueError(f"unknown job kind {self.kind!r}")


def _kerr_grid(rng):
    return int(rng.choice(KERR_N1)), int(rng.choice(KERR_N2)), int(rng.choice(KERR_N3))


def many_jobs(n_jobs=64, seed=3):
    """The fixed mix: the first half boxes, the second half Bondi flows."""
    rng = np.random.default_rng(seed)
    jobs = []
    for m in range(n_jobs):
        if m < n_jobs // 2:
            n = int(rng.choice(BOX_N))
            jobs.append(JobSpec(m, "box", n, n, n))
        else:
            a = float(rng.uniform(0.0, 0.99))
            n1, n2, n3 = _kerr_grid(rng)
            jobs.append(JobSpec(m, "bondi", n1, n2, n3, a=a))
    return jobs


def poisson_stream(n_jobs=300, lam=20.0, seed=4, steps=(200, 2000)):
    """The arrival stream: exponential inter-arrival gaps of mean 1/lam."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for m in range(n_jobs):
        t += float(rng.exponential(1.0 / lam))
        kind = "torus" if rng.random() < 0.5 else "bondi"
        a = float(rng.uniform(0.0, 0.99))
        n1, n2, n3 = _kerr_grid(rng)
        nsteps = int(rng.integers(steps[0], steps[1] + 1))
        jobs.append(JobSpec(m, kind, n1, n2, n3, a=a, steps=nsteps, arrival=t))
    return jobs
