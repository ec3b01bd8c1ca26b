"""One problem split along x3 into several contexts that exchange halos.

This is the shape of the multi-device decomposition on one device: each part
is an ordinary context over its share of the x3 planes, with DIRICHLET x3
boundaries so that the library keeps whatever ghost planes the driver writes.
Per substep the driver fills the physical ghost zones of every part (x1, x2),
copies the three x3 ghost planes on each side from the neighbouring parts'
interior planes (periodic in x3, whole planes including their x1/x2 ghosts, as
the single-domain x3 fill does), runs the substep, and combines the parts'
per-direction maximum signal speeds into one Courant step. Face fluxes in the
transverse ghost layer, and with them every Flux-CT EMF on a part boundary,
are recomputed from the exchanged planes, so no flux or EMF is exchanged.

With the x3 extent split into parts whose zone width equals the whole
domain's bit for bit (power-of-two splits of a power-of-two-scaled extent),
the split run reproduces the single-context run bit for bit, except where the
fixup repairs a zone next to a part boundary (it only averages neighbours that
its own part holds as interior).
"""

from ._binding import Sim, grmhd_fill_ghosts, grmhd_substep, grmhd_speeds, NG

BC_PERIODIC, BC_DIRICHLET = 0, 3


class SlabSplit:
    def __init__(self, prm, P0, parts, device="cuda:0"):
        n3 = prm["n3"]
        if n3 % parts:
            raise ValueError("n3 must be a multiple of the number of parts")
        if list(prm["bc"][2]) != [BC_PERIODIC, BC_PERIODIC]:
            raise ValueError("the split needs a periodic x3 direction")
        m = n3 // parts
        if m < NG:
            raise ValueError(f"each part needs at least {NG} x3 planes")
        dx3 = (prm["x3max"] - prm["x3min"]) / n3
        for i in range(parts):
            lo = prm["x3min"] + i * m * dx3
            hi = prm["x3min"] + (i + 1) * m * dx3
            if (hi - lo) / m != dx3:
                raise ValueError("a part's x3 zone width would differ from the domain's in the last bit")
        self.prm = prm
        self.parts = parts
        self.m = m
        self.sims, self.P, self.Ph = [], [], []
        for i in range(parts):
            sub = dict(prm)
            sub["n3"] = m
            sub["x3min"] = prm["x3min"] + i * m * dx3
            sub["x3max"] = prm["x3min"] + (i + 1) * m * dx3
            sub["bc"] = [list(prm["bc"][0]), list(prm["bc"][1]), [BC_DIRICHLET, BC_DIRICHLET]]
            sim = Sim(sub, device=device)
            self.sims.append(sim)
            self.P.append(sim.to_device(P0[:, i * m:(i + 1) * m + 2 * NG]))
            self.Ph.append(sim.empty_state())
        self.dx = [(prm["x1max"] - prm["x1min"]) / prm["n1"], (prm["x2max"] - prm["x2min"]) / prm["n2"], dx3]

    def exchange(self, states):
        """x3 ghost planes of every part from its neighbours' interior planes."""
        m, n = self.m, self.parts
        for i in range(n):
            below, above = states[(i - 1) % n], states[(i + 1) % n]
            states[i][:, 0:NG] = below[:, m:m + NG]
            states[i][:, m + NG:m + 2 * NG] = above[:, NG:2 * NG]

    def step(self, dt):
        """One predictor-corrector step of every part; returns the Courant step
        for the next one from the corrector's speeds over the whole domain."""
        for s, P in zip(self.sims, self.P):
            grmhd_fill_ghosts(s.ctx, P, None)
        self.exchange(self.P)
        for s, P, Ph in zip(self.sims, self.P, self.Ph):
            grmhd_substep(s.ctx, P, P, Ph, 0.5 * dt, False)
        for s, P, Ph in zip(self.sims, self.P, self.Ph):
            grmhd_fill_ghosts(s.ctx, Ph, P)
        self.exchange(self.Ph)
        for s, P, Ph in zip(self.sims, self.P, self.Ph):
            grmhd_substep(s.ctx, Ph, P, P, dt, True)
        vmax = [0.0, 0.0, 0.0]
        for s in self.sims:
            v = grmhd_speeds(s.ctx)
            vmax = [max(a, b) for a, b in zip(vmax, v)]
        total = 0.0
        for d in range(3):
            total += vmax[d] / self.dx[d]
        return self.prm["cfl"] / total if total > 0.0 else float("inf")

    def to_host(self):
        """The whole interior [8, n3, n2, n1] assembled from the parts."""
        import numpy as np
        out = []
        for s, P in zip(self.sims, self.P):
            out.append(s.interior(P).cpu().numpy())
        return np.concatenate(out, axis=1)

    def close(self):
        for s in self.sims:
            s.close()
        self.sims = []
