"""One problem split along x3 into several contexts that exchange halos.

This is the shape of the multi-device decomposition on one device: each part
is an ordinary context over its share of the x3 planes, with DIRICHLET x3
boundaries so that the library keeps whatever ghost planes the driver writes.
Per substep the driver fills the physical ghost zones of every part (x1, x2),
copies the three x3 ghost planes on each side from the neighbouring parts'
interior planes (periodic in x3, whole planes including their x1/x2 ghosts, as
the single-domain x3 fill does), runs the update of every part
(grmhd_update), copies each part's new boundary planes and their failure flags
into its neighbours' first ghost planes, runs the fixup of every part with its
two x3 sides as halo sides (grmhd_fixup), and combines the parts'
per-direction maximum signal speeds into one Courant step
(grmhd_courant_dt). Face fluxes in the transverse ghost layer, and with them
every Flux-CT EMF on a part boundary, are recomputed from the exchanged
planes, so no flux or EMF is exchanged; a failed zone next to a part boundary
is repaired from the same 26 neighbours as in the undivided domain.

With the x3 extent split into parts whose zone width equals the whole
domain's bit for bit (power-of-two splits of a power-of-two-scaled extent),
the split run reproduces the single-context run bit for bit.
"""

from ._binding import (Sim, grmhd_fill_ghosts, grmhd_update, grmhd_fixup, grmhd_speeds, grmhd_courant_dt,
                       NG)

HALO_X3 = (1 << 4) | (1 << 5)          # both x3 sides of a part hold neighbour zones

BC_PERIODIC, BC_DIRICHLET = 0, 3
KERR_CKS = 3


class SlabSplit:
    def __init__(self, prm, P0, parts, device="cuda:0"):
        n3 = prm["n3"]
        if n3 % parts:
            raise ValueError("n3 must be a multiple of the number of parts")
        if list(prm["bc"][2]) != [BC_PERIODIC, BC_PERIODIC]:
            raise ValueError("the split needs a periodic x3 direction")
        if prm["coords"] == KERR_CKS:
            # each part builds its own tables from its own x3 extent; where the
            # geometry depends on x3 those would match the whole domain's only
            # to rounding, and the centred-difference connection magnifies that
            raise ValueError("the split needs geometry that does not depend on x3")
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
        self.sims, self.P, self.Ph, self.flags = [], [], [], []
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
            self.flags.append(sim.torch.zeros(tuple(sim.shape[1:]), dtype=sim.torch.int8, device=sim.device))

    def exchange(self, states):
        """x3 ghost planes of every part from its neighbours' interior planes."""
        m, n = self.m, self.parts
        for i in range(n):
            below, above = states[(i - 1) % n], states[(i + 1) % n]
            states[i][:, 0:NG] = below[:, m:m + NG]
            states[i][:, m + NG:m + 2 * NG] = above[:, NG:2 * NG]

    def exchange_boundary(self, states):
        """The first x3 ghost plane of every part (values and failure flags)
        from its neighbours' boundary interior planes, for the fixup."""
        m, n = self.m, self.parts
        for arrs in (states, self.flags):
            for i in range(n):
                below, above = arrs[(i - 1) % n], arrs[(i + 1) % n]
                arrs[i][..., NG - 1, :, :] = below[..., m + NG - 1, :, :]
                arrs[i][..., m + NG, :, :] = above[..., NG, :, :]

    def substep(self, Ps, Pb, Pout, dt, want_speeds):
        for s, a, b, c, f in zip(self.sims, Ps, Pb, Pout, self.flags):
            grmhd_update(s.ctx, a, b, c, dt, f, want_speeds)
        self.exchange_boundary(Pout)
        for s, c, f in zip(self.sims, Pout, self.flags):
            grmhd_fixup(s.ctx, c, f, HALO_X3)

    def step(self, dt):
        """One predictor-corrector step of every part; returns the Courant step
        for the next one from the corrector's speeds over the whole domain."""
        for s, P in zip(self.sims, self.P):
            grmhd_fill_ghosts(s.ctx, P, None)
        self.exchange(self.P)
        self.substep(self.P, self.P, self.Ph, 0.5 * dt, False)
        for s, P, Ph in zip(self.sims, self.P, self.Ph):
            grmhd_fill_ghosts(s.ctx, Ph, P)
        self.exchange(self.Ph)
        self.substep(self.Ph, self.P, self.P, dt, True)
        return grmhd_courant_dt(self.sims[0].ctx, [grmhd_speeds(s.ctx) for s in self.sims])

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
