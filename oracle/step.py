"""Boundaries, fluxes, Flux-CT, update, bounds, time step and driver (oracle).

Functionality section: HARM updates conserved variables by finite volumes
on a mesh that is uniform in its code coordinates. One step of the method, as this oracle evaluates it
(the paper defers the scheme to the HARM papers; the readings are stated where
they are taken):

  predictor  U_h    = U(P^n) + dt/2 L(P^n),    P_h    = invert(U_h; guess P^n)
  corrector  U^n+1  = U(P^n) + dt   L(P_h),    P^n+1  = invert(U^n+1; guess P_h)
  L(P) = -sum_d [F_d(i + e_d) - F_d(i)] / dx_d + S(P)

with face fluxes from reconstructed primitives and a local Lax-Friedrichs
flux, Flux-CT for the magnetic field (Implementation Notes: Toth 2000), the
geometric source S_nu = sqrt(-g) T^k_l Gamma^l_{nu k}, and the bounds of the
Implementation Notes applied after every substep (reading: "at the end of each
step" taken per substep so the corrector never sees an unbounded state).
"""

import numpy as np

from .grid import NG
from .physics import fluid_state, flux, conserved, signal_speeds, stress
from .recon import reconstruct
from .invert import invert

BC_PERIODIC, BC_OUTFLOW, BC_POLAR, BC_DIRICHLET = 0, 1, 2, 3
B1, B2, B3 = 5, 6, 7
GROWTH = 1.3


# ----------------------------------------------------------------------------- helpers

def _interior(n3, n2, n1):
    return (slice(None), slice(NG, NG + n3), slice(NG, NG + n2), slice(NG, NG + n1))




# ----------------------------------------------------------------------------- boundaries

def _inflow_fix(P, geo, side):
    """Outflow ghost whose radial four-velocity points into the domain: reset
    u~1 so that u^1 = 0 (reading of the silent radial boundary).

    With c = alpha g^{t1}, u^1 = 0 means u~1 = c Gamma, and Gamma is the positive
    root of (1 - g_11 c^2) G^2 - 2 c (g_12 u~2 + g_13 u~3) G - (1 + g_jk u~j u~k) = 0
    (j, k in {2, 3}); where that quadratic has no positive leading coefficient the
    ghost is left alone.
    """
    gcov, gcon, alpha = geo["gcov"], geo["gcon"], geo["alpha"]
    v1, v2, v3 = P[2], P[3], P[4]
    lor = np.sqrt(1.0 + sum(gcov[i + 1, j + 1] * P[2 + i] * P[2 + j]
                            for i in range(3) for j in range(3)))
    u1 = v1 - lor * alpha * gcon[0, 1]
    bad = (u1 > 0.0) if side == 0 else (u1 < 0.0)
    c = alpha * gcon[0, 1]
    qa = 1.0 - gcov[1, 1] * c * c
    G = gcov[1, 2] * v2 + gcov[1, 3] * v3
    H = gcov[2, 2] * v2 * v2 + 2.0 * gcov[2, 3] * v2 * v3 + gcov[3, 3] * v3 * v3
    with np.errstate(all="ignore"):
        root = (c * G + np.sqrt(c * c * G * G + qa * (1.0 + H))) / qa
    fix = bad & (qa > 0.0)
    P[2] = np.where(fix, c * root, v1)


def fill_ghosts(P, grid, do_x3=True):
    """Fill the ghost zones of a padded primitive array in place.

    Order: x1 (interior j, k), then x2 (all i, interior k), then x3 (all i, j).
    Periodic: wrap. Outflow (x1 only): copy the nearest interior zone, then the
    inflow check. Polar (x2 only): ghost row -1-m mirrors row m with u~2 and B2
    negated. Dirichlet: the ghosts keep the values they hold.
    With ``do_x3=False`` the x3 ghosts are taken to be real neighbour data (a
    window of a larger domain) and are left alone.
    """
    prm = grid.prm
    n1, n2 = grid.n[0], grid.n[1]
    nk = P.shape[1] - 2 * NG
    bc = prm["bc"]
    K = slice(NG, NG + nk)
    J = slice(NG, NG + n2)
    # x1
    for side in (0, 1):
        t = bc[0][side]
        for m in range(NG):
            g = NG - 1 - m if side == 0 else NG + n1 + m
            if t == BC_PERIODIC:
                s = NG + n1 - 1 - m if side == 0 else NG + m
            elif t == BC_OUTFLOW:
                s = NG if side == 0 else NG + n1 - 1
            elif t == BC_DIRICHLET:
                continue
            else:
                raise ValueError("unsupported x1 boundary")
            P[:, K, J, g] = P[:, K, J, s]
        if t == BC_OUTFLOW:
            gs = slice(0, NG) if side == 0 else slice(NG + n1, NG + n1 + NG)
            sub = P[:, K, J, gs]
            _inflow_fix(sub, grid.sub(grid.cent, K, J, gs), side)
            P[:, K, J, gs] = sub
    # x2
    for side in (0, 1):
        t = bc[1][side]
        for m in range(NG):
            g = NG - 1 - m if side == 0 else NG + n2 + m
            if t == BC_PERIODIC:
                s = NG + n2 - 1 - m if side == 0 else NG + m
            elif t == BC_POLAR:
                s = NG + m if side == 0 else NG + n2 - 1 - m
            elif t == BC_OUTFLOW:
                s = NG if side == 0 else NG + n2 - 1
            elif t == BC_DIRICHLET:
                continue
            P[:, K, g, :] = P[:, K, s, :]
            if t == BC_POLAR:
                P[3, K, g, :] *= -1.0
                P[B2, K, g, :] *= -1.0
    # x3
    if do_x3:
        n3 = grid.n[2]
        for side in (0, 1):
            t = bc[2][side]
            for m in range(NG):
                g = NG - 1 - m if side == 0 else NG + n3 + m
                if t == BC_PERIODIC:
                    s = NG + n3 - 1 - m if side == 0 else NG + m
                elif t == BC_OUTFLOW:
                    s = NG if side == 0 else NG + n3 - 1
                elif t == BC_DIRICHLET:
                    continue
                else:
                    raise ValueError("unsupported x3 boundary")
                P[:, g, :, :] = P[:, s, :, :]
    return P


# ----------------------------------------------------------------------------- fluxes

AXIS = {1: 3, 2: 2, 3: 1}


def face_fluxes(P, grid, d):
    """LLF fluxes at the lower d-faces of every zone with a full stencil.

    Returns (F, ctop) on the padded index grid of ``P``; faces 0..n_d along d
    (padded NG..NG+n_d) are filled for every transverse index, the rest is NaN.
    At an outflow boundary in x1 the rest-mass flux is clipped so that no mass
    enters the domain.

    F = (F_L + F_R)/2 - ctop (U_R - U_L)/2,  ctop = max(c_max, c_min) with
    c_max = max(0, c+_L, c+_R), c_min = max(0, -c-_L, -c-_R).
    """
    prm = grid.prm
    gam = prm["gam"]
    ax = AXIS[d]
    n = P.shape[ax] - 2 * NG
    f0, f1 = NG, NG + n + 1
    PL, PR = reconstruct(P, ax, prm["recon"], f0, f1)
    sl = [slice(None)] * 3                 # (k, j, i) of the face table
    sl[ax - 1] = slice(f0, f1)
    geo = grid.sub(grid.face[d], *sl)
    gdet = geo["gdet"]
    sL = fluid_state(PL, geo, gam)
    sR = fluid_state(PR, geo, gam)
    FL, FR = flux(sL, d, gdet), flux(sR, d, gdet)
    UL, UR = conserved(sL, gdet), conserved(sR, gdet)
    cpL, cmL = signal_speeds(sL, geo, d, gam)
    cpR, cmR = signal_speeds(sR, geo, d, gam)
    cmax = np.maximum(np.maximum(0.0, cpL), cpR)
    cmin = np.maximum(np.maximum(0.0, -cmL), -cmR)
    ctop = np.maximum(cmax, cmin)
    Fface = 0.5 * (FL + FR) - 0.5 * ctop * (UR - UL)
    if d == 1:
        # reading of the silent radial boundary: no mass enters through an
        # outflow boundary, so the rest-mass flux through the inner radial face
        # is at most 0 and through the outer one at least 0
        bc = prm["bc"][0]
        if bc[0] == BC_OUTFLOW:
            Fface[0, ..., 0] = np.minimum(Fface[0, ..., 0], 0.0)
        if bc[1] == BC_OUTFLOW:
            Fface[0, ..., -1] = np.maximum(Fface[0, ..., -1], 0.0)
    F = np.full(P.shape, np.nan)
    C = np.full(P.shape[1:], np.nan)
    sl = [slice(None)] * 4
    sl[ax] = slice(f0, f1)
    F[tuple(sl)] = Fface
    C[tuple(sl[1:])] = ctop
    return F, C


def flux_ct(F1, F2, F3, grid):
    """Flux-CT (Implementation Notes: Toth 2000), in place.

    Edge EMFs from the four face fluxes around each edge,
      emf3(i,j,k) = [F1_B2(i,j) + F1_B2(i,j-1) - F2_B1(i,j) - F2_B1(i-1,j)]/4
      emf1(i,j,k) = [F2_B3(j,k) + F2_B3(j,k-1) - F3_B2(j,k) - F3_B2(j-1,k)]/4
      emf2(i,j,k) = [F3_B1(i,k) + F3_B1(i-1,k) - F1_B3(i,k) - F1_B3(i,k-1)]/4
    replace the face B fluxes by averages of the two edge EMFs bounding the face,
    which keeps the corner-centred divergence of sqrt(-g) B unchanged.
    Reading for polar boundaries: the EMFs on the axis edges are zero (they
    vanish by the reflection symmetry), and the hydrodynamic x2 fluxes through
    the axis faces are zero.
    """
    prm = grid.prm
    n2 = grid.n[1]
    nan = np.nan
    e3 = np.full(F1.shape[1:], nan)
    e1 = np.full(F1.shape[1:], nan)
    e2 = np.full(F1.shape[1:], nan)
    e3[:, 1:, 1:] = 0.25 * (F1[B2, :, 1:, 1:] + F1[B2, :, :-1, 1:] - F2[B1, :, 1:, 1:] - F2[B1, :, 1:, :-1])
    e1[1:, 1:, :] = 0.25 * (F2[B3, 1:, 1:, :] + F2[B3, :-1, 1:, :] - F3[B2, 1:, 1:, :] - F3[B2, 1:, :-1, :])
    e2[1:, :, 1:] = 0.25 * (F3[B1, 1:, :, 1:] + F3[B1, 1:, :, :-1] - F1[B3, 1:, :, 1:] - F1[B3, :-1, :, 1:])
    for side, t in enumerate(prm["bc"][1]):
        if t == BC_POLAR:
            jf = NG if side == 0 else NG + n2
            e1[:, jf, :] = 0.0
            e3[:, jf, :] = 0.0
            F2[0:5, :, jf, :] = 0.0
    F1[B1] = 0.0
    F1[B2, :, :-1, :] = 0.5 * (e3[:, :-1, :] + e3[:, 1:, :])
    F1[B3, :-1, :, :] = -0.5 * (e2[:-1, :, :] + e2[1:, :, :])
    F2[B1, :, :, :-1] = -0.5 * (e3[:, :, :-1] + e3[:, :, 1:])
    F2[B2] = 0.0
    F2[B3, :-1, :, :] = 0.5 * (e1[:-1, :, :] + e1[1:, :, :])
    F3[B1, :, :, :-1] = 0.5 * (e2[:, :, :-1] + e2[:, :, 1:])
    F3[B2, :, :-1, :] = -0.5 * (e1[:, :-1, :] + e1[:, 1:, :])
    F3[B3] = 0.0


# ----------------------------------------------------------------------------- source, bounds

def source(P, geo, conn, gam):
    """S_nu = sqrt(-g) T^k_l Gamma^l_{nu k} for nu = t..3, [4, ...]."""
    st = fluid_state(P, geo, gam)
    T = [[stress(st, k, l) for l in range(4)] for k in range(4)]
    S = []
    for nu in range(4):
        S.append(geo["gdet"] * sum(T[k][l] * conn[l, nu, k] for k in range(4) for l in range(4)))
    return np.array(np.broadcast_arrays(*S))


def floors(P, geo, r, prm, mask=None):
    """The bounds of the Implementation Notes, in primitive space, in place.

    Reading of "incremented"/"downscaled" (order and frame are not given):
    1. if Gamma > gamma_max, scale u~ by sqrt((gamma_max^2 - 1)/(Gamma^2 - 1));
    2. with b^2 from the rescaled state,
       rho <- max(rho, rho_fl k, b^2/sigma_max)          (sigma = b^2/rho < sigma_max)
    3. u   <- max(u, u_fl k^gamma, beta_min b^2 / (2 (gamma-1)))  (beta = p_gas/(b^2/2))
    4. rho <- max(rho, u / uorho_max)
    with k = 1/(r^2 (1 + r/10)). ``mask`` restricts the update to some zones.
    """
    gam = prm["gam"]
    gcov = geo["gcov"]
    v = P[2:5]
    lor2 = 1.0 + sum(gcov[i + 1, j + 1] * v[i] * v[j] for i in range(3) for j in range(3))
    gmax = prm["gamma_max"]
    with np.errstate(all="ignore"):
        scale = np.where(lor2 > gmax * gmax, np.sqrt((gmax * gmax - 1.0) / (lor2 - 1.0)), 1.0)
    new = P.copy()
    new[2:5] = v * scale
    st = fluid_state(new, geo, gam)
    bsq = st["bsq"]
    k = 1.0 / (r * r * (1.0 + r / 10.0))
    rho = np.maximum(np.maximum(new[0], prm["rho_fl"] * k), bsq / prm["sigma_max"])
    u = np.maximum(np.maximum(new[1], prm["u_fl"] * k ** gam),
                   prm["beta_min"] * bsq / (2.0 * (gam - 1.0)))
    rho = np.maximum(rho, u / prm["uorho_max"])
    new[0] = rho
    new[1] = u
    if mask is None:
        P[:] = new
    else:
        P[:] = np.where(mask, new, P)
    return P


def _neighbour(a, off, wrap, fill):
    """b[x] = a[x + off] over the last three axes (k, j, i); an axis with
    wrap[axis] True is periodic, otherwise out-of-range entries are ``fill``."""
    b = a
    for ax, (o, w) in enumerate(zip(off, wrap)):
        if o == 0:
            continue
        axis = b.ndim - 3 + ax
        if w:
            b = np.roll(b, -o, axis=axis)
        else:
            n = b.shape[axis]
            out = np.full_like(b, fill)
            src = [slice(None)] * b.ndim
            dst = [slice(None)] * b.ndim
            src[axis] = slice(max(0, o), n + min(0, o))
            dst[axis] = slice(max(0, -o), n - max(0, o))
            out[tuple(dst)] = b[tuple(src)]
            b = out
    return b


def fixup(P, failed, wrap=(False, False, False)):
    """Repair zones whose inversion failed, in place.

    Reading (the paper only says the bounds avoid catastrophic failures): a
    failed zone takes the mean of the hydrodynamic primitives (rho, u, u~) of
    its non-failed neighbours among the 26 around it, read from the array
    before any repair; with none it keeps what it holds. B is never touched
    (it comes straight from U). Neighbours are taken across periodic
    directions (``wrap``, in (x3, x2, x1) = array axis order), so the repair
    of a zone does not depend on where the periodic seam of the domain lies
    (or, for a domain split into parts, on where the part boundaries lie);
    across a non-periodic edge there are no neighbours.
    """
    if not failed.any():
        return P
    ok = ~failed
    acc = np.zeros((5,) + failed.shape)
    cnt = np.zeros(failed.shape)
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                if dk == dj == di == 0:
                    continue
                w = _neighbour(ok, (dk, dj, di), wrap, False)
                acc += np.where(w, _neighbour(P[:5], (dk, dj, di), wrap, 0.0), 0.0)
                cnt += w
    fix = failed & (cnt > 0)
    with np.errstate(all="ignore"):
        P[:5] = np.where(fix, acc / cnt, P[:5])
    return P


def periodic_axes(prm, window=False):
    """(x3, x2, x1) periodicity of a block for the fixup; a window of x3 planes
    cut from a larger domain is not periodic in x3."""
    per = [prm["bc"][d][0] == BC_PERIODIC for d in range(3)]
    return (per[2] and not window, per[1], per[0])


# ----------------------------------------------------------------------------- substep / step

def substep(Ps, Pb, grid, dt, mass_flux=False, window=False):
    """One substep on a padded block.

    Ps: flux-state primitives with ghosts filled (padded block); Pb: base-state
    primitives on the block interior. Returns (P_new interior, failed mask,
    ctop maxima per direction over the interior faces), and with
    ``mass_flux`` also the three mass-flux arrays (component 0 of the face
    fluxes after Flux-CT, padded grid). ``window``: the block is a window of x3
    planes of a larger domain (its fixup does not wrap in x3).
    """
    prm = grid.prm
    gam = prm["gam"]
    nk = Ps.shape[1] - 2 * NG
    n1, n2 = grid.n[0], grid.n[1]
    if grid.k3 and nk != grid.n[2]:
        raise ValueError("3D geometry tables need the whole x3 extent")
    F1, C1 = face_fluxes(Ps, grid, 1)
    F2, C2 = face_fluxes(Ps, grid, 2)
    F3, C3 = face_fluxes(Ps, grid, 3)
    flux_ct(F1, F2, F3, grid)
    K, J, I = slice(NG, NG + nk), slice(NG, NG + n2), slice(NG, NG + n1)
    Kp, Jp, Ip = slice(NG + 1, NG + nk + 1), slice(NG + 1, NG + n2 + 1), slice(NG + 1, NG + n1 + 1)
    dx1, dx2, dx3 = grid.dx
    div = ((F1[:, K, J, Ip] - F1[:, K, J, I]) / dx1 + (F2[:, K, Jp, I] - F2[:, K, J, I]) / dx2
           + (F3[:, Kp, J, I] - F3[:, K, J, I]) / dx3)
    geo = grid.sub(grid.cent, K, J, I)
    conn = grid.sub(grid.conn, K, J, I)
    r = grid.sub(grid.r, K, J, I) if grid.kerr else None
    Psi = Ps[:, K, J, I]
    S = source(Psi, geo, conn, gam)
    U0 = conserved(fluid_state(Pb, geo, gam), geo["gdet"])
    rhs = -div
    rhs[1:5] += S
    Ustar = U0 + dt * rhs
    Pn, failed = invert(Ustar, Psi, geo, gam)
    if prm["floors"]:
        floors(Pn, geo, r, prm)
    if failed.any():
        fixup(Pn, failed, periodic_axes(prm, window))
        if prm["floors"]:
            floors(Pn, geo, r, prm, mask=failed)
    cmax = (np.nanmax(C1[K, J, NG:NG + n1 + 1]), np.nanmax(C2[K, NG:NG + n2 + 1, I]),
            np.nanmax(C3[NG:NG + nk + 1, J, I]))
    if mass_flux:
        return Pn, failed, cmax, (F1[0], F2[0], F3[0])
    return Pn, failed, cmax


def dt_from_ctop(cmax, grid):
    """Courant step dt = cfl / sum_d (max ctop_d / dx_d) (reading of the CFL rule)."""
    return grid.prm["cfl"] / sum(c / dx for c, dx in zip(cmax, grid.dx))


def step(P, grid, dt):
    """One predictor-corrector step of a padded state. Returns (P_new, dt_next, info)."""
    n1, n2, n3 = grid.n
    it = _interior(n3, n2, n1)
    P0 = fill_ghosts(P.copy(), grid)
    Ph_i, f1, _ = substep(P0, P0[it], grid, 0.5 * dt)
    Ph = P0.copy()
    Ph[it] = Ph_i
    fill_ghosts(Ph, grid)
    Pn_i, f2, cmax = substep(Ph, P0[it], grid, dt)
    Pn = P0.copy()
    Pn[it] = Pn_i
    info = dict(fail_predictor=int(f1.sum()), fail_corrector=int(f2.sum()), ctop=cmax)
    return Pn, dt_from_ctop(cmax, grid), info


def get_dt(P, grid):
    """Courant dt of state P from its own face signal speeds."""
    n1, n2, n3 = grid.n
    Q = fill_ghosts(P.copy(), grid)
    K, J, I = slice(NG, NG + n3), slice(NG, NG + n2), slice(NG, NG + n1)
    C1 = face_fluxes(Q, grid, 1)[1]
    C2 = face_fluxes(Q, grid, 2)[1]
    C3 = face_fluxes(Q, grid, 3)[1]
    cmax = (np.nanmax(C1[K, J, NG:NG + n1 + 1]), np.nanmax(C2[K, NG:NG + n2 + 1, I]),
            np.nanmax(C3[NG:NG + n3 + 1, J, I]))
    return dt_from_ctop(cmax, grid)


def run(P, grid, nsteps, dt=None):
    """Evolve nsteps with dt <- min(dt_next, 1.3 dt). Returns (P, [dt used per step])."""
    if dt is None:
        dt = get_dt(P, grid)
    used = []
    for _ in range(nsteps):
        used.append(dt)
        P, dt_next, _ = step(P, grid, dt)
        dt = min(dt_next, GROWTH * dt)
    return P, used


def step_window(P, grid, dt, k0, k1):
    """P^{n+1} on interior slabs k0..k1-1 of a full padded state, computed from a
    window of x3 slabs around them (x1 and x2 cover the whole domain).

    The window is wide enough that every value it returns equals the full-domain
    step: 8 slabs of margin per side (3 per substep for the stencil and CT plus
    1 per substep so that fixups never read outside the window).
    """
    n1, n2, n3 = grid.n
    full = fill_ghosts(P.copy(), grid)
    M1 = 5
    ks = np.arange(k0 - M1 - NG, k1 + M1 + NG) % n3 + NG
    blk = full[:, ks]
    it1 = (slice(None), slice(NG, blk.shape[1] - NG), slice(NG, NG + n2), slice(NG, NG + n1))
    Ph_i, _, _ = substep(blk, blk[it1], grid, 0.5 * dt, window=True)
    ph = blk.copy()
    ph[it1] = Ph_i
    fill_ghosts(ph, grid, do_x3=False)
    # substep 2 block: P_h slabs k0-1-NG .. k1+1+NG  (interior k0-1 .. k1+1)
    off = (M1 + NG) - (1 + NG)
    blk2 = ph[:, off:off + (k1 - k0) + 2 + 2 * NG]
    base = blk[:, off + NG:off + NG + (k1 - k0) + 2, NG:NG + n2, NG:NG + n1]
    Pn_i, _, _ = substep(blk2, base, grid, dt, window=True)
    return Pn_i[:, 1:-1]


# ----------------------------------------------------------------------------- pointwise calls

def prim_to_cons(P, grid):
    """U on the interior zones of a padded primitive array."""
    n1, n2, n3 = grid.n
    it = _interior(n3, n2, n1)
    geo = grid.sub(grid.cent, *it[1:])
    return conserved(fluid_state(P[it], geo, grid.prm["gam"]), geo["gdet"])


def cons_to_prim(U, guess, grid, do_floors=True, do_fixup=True):
    """Invert interior conserved variables (then bounds and fixup)."""
    n1, n2, n3 = grid.n
    K, J, I = slice(NG, NG + n3), slice(NG, NG + n2), slice(NG, NG + n1)
    geo = grid.sub(grid.cent, K, J, I)
    r = grid.sub(grid.r, K, J, I) if grid.kerr else None
    P, failed = invert(U, guess, geo, grid.prm["gam"])
    if do_floors and grid.prm["floors"]:
        floors(P, geo, r, grid.prm)
    if do_fixup and failed.any():
        fixup(P, failed, periodic_axes(grid.prm))
        if do_floors and grid.prm["floors"]:
            floors(P, geo, r, grid.prm, mask=failed)
    return P, failed


def divb(P, grid):
    """max |div B| over corners, corner-centred divergence of sqrt(-g) B.

    At corner (i-1/2, j-1/2, k-1/2):
      divB = sum_d 1/(4 dx_d) sum_{a,b in {0,1}} [G_d(+ side) - G_d(- side)],
    G_d = sqrt(-g) B^d at zone centres, the transverse offsets a, b running over
    the two zones on each side. Corners on non-periodic boundaries are excluded;
    periodic directions wrap.
    """
    prm = grid.prm
    n1, n2, n3 = grid.n
    it = _interior(n3, n2, n1)
    gd = grid.sub(grid.cent["gdet"], *it[1:])
    G = [P[it][B1 + d] * gd for d in range(3)]
    per = [prm["bc"][d][0] == BC_PERIODIC for d in range(3)]

    def sh(a, s, ax):  # value at index (i - s) along axis ax, periodic wrap
        return np.roll(a, s, axis=ax)

    dx1, dx2, dx3 = grid.dx
    # axes of [k, j, i]: 2 = i (x1), 1 = j (x2), 0 = k (x3)
    def corner_sum(a, ax_t1, ax_t2):
        return a + sh(a, 1, ax_t1) + sh(a, 1, ax_t2) + sh(sh(a, 1, ax_t1), 1, ax_t2)

    d1 = corner_sum(G[0] - sh(G[0], 1, 2), 1, 0) / (4 * dx1)
    d2 = corner_sum(G[1] - sh(G[1], 1, 1), 2, 0) / (4 * dx2)
    d3 = corner_sum(G[2] - sh(G[2], 1, 0), 2, 1) / (4 * dx3)
    div = d1 + d2 + d3
    sl = tuple(slice(0 if per[ax] else 1, None) for ax in (2, 1, 0))
    return float(np.max(np.abs(div[sl]))) if div[sl].size else 0.0
