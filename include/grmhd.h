/*
 * grmhd.h -- C ABI of an MI355X (gfx950) library that advances ideal
 * general-relativistic MHD in a fixed stationary spacetime by the HARM
 * conservative finite-volume scheme that iharm3D implements.
 *
 * What the calls compute (the problem as the paper states it):
 *   - ideal GRMHD on a mesh uniform in code coordinates (any coordinates) of a
 *     stationary metric whose line element is analytic (Functionality section;
 *     Implementation Notes: metric quantities evaluated numerically);
 *   - units GM = c = 1 (Implementation Notes);
 *   - conserved variables stepped in time and inverted to primitives by the
 *     1D_W scheme (Implementation Notes, after Noble et al. 2006);
 *   - Flux-CT transport of the magnetic field (Implementation Notes, after
 *     Toth 2000);
 *   - the density / energy / magnetisation / Lorentz-factor bounds of the
 *     Implementation Notes, applied after every substep.
 *
 * Data layout. A state (primitive P or conserved U) is one float64 array
 *   [8][n3 + 6][n2 + 6][n1p],   n1p = n1 + 6 rounded up to a multiple of 8,
 * x1 fastest, 3 ghost layers on each side of each direction; interior zone
 * (i, j, k) sits at element ((v*(n3+6) + k+3)*(n2+6) + j+3)*n1p + i+3.
 * grmhd_state_layout() returns the shape and strides. Variables, in order:
 *   P: rho, u (internal energy density), u~1, u~2, u~3 (velocity relative to
 *      the normal observer, code coordinates), B1, B2, B3;
 *   U: sqrt(-g) (rho u^t, T^t_t + rho u^t, T^t_1, T^t_2, T^t_3, B1, B2, B3).
 * Elements in the x1 alignment padding (i >= n1 + 3) are never read.
 *
 * Ownership and streams. The caller owns every state buffer: device memory on
 * the device current at grmhd_init, sized per grmhd_state_layout. The library
 * owns its geometry tables and scratch from grmhd_init until grmhd_free and
 * keeps no caller pointer after a call returns. All work is enqueued on the
 * stream given to grmhd_init; a call that returns a host scalar (dt, dt_next,
 * n_fail, max_divb) synchronises that stream, every other call is
 * asynchronous. Calls on one context must not overlap from several host
 * threads.
 *
 * Errors. Every call returns GRMHD_OK (0) or a negative grmhd_status and
 * never throws; grmhd_last_error(ctx) gives a message for the last failure on
 * that context. Inversion failures are not errors: they are flagged per zone
 * and repaired by the fixup (the bounds exist "to avoid catastrophic
 * failures", Implementation Notes).
 */
#ifndef GRMHD_H
#define GRMHD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GRMHD_OK = 0,
  GRMHD_EINVAL = -1,       /* bad argument: null pointer, bad size or enum */
  GRMHD_ENOMEM = -2,       /* device allocation failed */
  GRMHD_EDEVICE = -3,      /* HIP runtime / kernel launch error, or no device */
  GRMHD_EUNSUPPORTED = -4, /* valid but not implemented combination */
  GRMHD_ESTATE = -5        /* a non-finite value appeared in the evolved state */
} grmhd_status;

enum { GRMHD_MINKOWSKI_CART = 0, GRMHD_KERR_MKS = 1, GRMHD_KERR_FMKS = 2, GRMHD_KERR_CKS = 3 };
enum { GRMHD_RECON_MC = 0, GRMHD_RECON_WENO5 = 1 };
enum { GRMHD_FP64 = 0, GRMHD_MIXED = 1 };
enum { GRMHD_BC_PERIODIC = 0, GRMHD_BC_OUTFLOW = 1, GRMHD_BC_POLAR = 2, GRMHD_BC_DIRICHLET = 3 };
enum { GRMHD_OPT_FLOORS = 1, GRMHD_OPT_FIXUP = 2 };

/* Only the calls below are exported from the shared library. */
#define GRMHD_API __attribute__((visibility("default")))

#define GRMHD_NG 3
#define GRMHD_NVAR 8
#define GRMHD_NSCALAR 2

/* One problem. Code coordinates:
 *   MINKOWSKI_CART: Cartesian, metric diag(-1, 1, 1, 1);
 *   KERR_MKS:  Kerr-Schild with r = exp(x1), theta = pi x2 + (1-hslope)/2 sin(2 pi x2),
 *              phi = x3;
 *   KERR_FMKS: as MKS, with theta blended towards the polynomial
 *              theta_J = N y (1 + (y/poly_xt)^poly_alpha/(poly_alpha+1)) + pi/2,
 *              y = 2 x2 - 1, by exp(-mks_smooth (x1 - x1min)).
 *   KERR_CKS:  Cartesian Kerr-Schild, (x1, x2, x3) = (x, y, z), metric
 *              eta + f l l with f = 2 r^3/(r^4 + a^2 z^2), l = (1, (r x + a y)/(r^2 + a^2),
 *              (r y - a x)/(r^2 + a^2), z/r) and r the positive root of
 *              r^4 - (x^2 + y^2 + z^2 - a^2) r^2 - a^2 z^2 = 0 (Implementation Notes:
 *              a change of coordinates or background spacetime). The metric
 *              depends on all three coordinates: the geometry tables are 3D
 *              (about 1.3 KB of device memory per zone, counted by
 *              grmhd_context_bytes; at most 2^25 zones, ghosts and x1
 *              padding included). Boundaries PERIODIC or DIRICHLET only; the
 *              box, ghosts included, must lie outside the unit sphere
 *              x^2 + y^2 + z^2 < 1 (so r > 0 and the metric is regular).
 * Zone centres sit at x_d = xdmin + (i + 1/2) (xdmax - xdmin)/nd.
 * bc[d][side]: boundary type of direction d (0 = x1) at its lower (0) / upper (1)
 * edge; PERIODIC on both sides or neither; OUTFLOW only in x1 of MKS / FMKS;
 * POLAR only in x2 of MKS / FMKS; DIRICHLET keeps the ghost values the caller
 * stored in the state.
 * floors: 1 applies the bounds (needs a Kerr metric: they use r). */
typedef struct grmhd_problem {
  int32_t n1, n2, n3;
  int32_t coords;
  double a, gam, cfl;
  double x1min, x1max, x2min, x2max, x3min, x3max;
  double hslope, poly_xt, poly_alpha, mks_smooth;
  int32_t recon;
  int32_t precision;
  int32_t bc[3][2];
  int32_t floors;
  double rho_fl, u_fl, sigma_max, beta_min, uorho_max, gamma_max;
} grmhd_problem;

typedef struct grmhd_ctx grmhd_ctx;

/* Validate the problem, build the geometry tables on the device (metric,
 * inverse, sqrt(-g), lapse at zone centres and faces; connection at centres by
 * centred differences) and allocate scratch. hip_stream: a hipStream_t, or NULL
 * for the null stream. Errors: EINVAL (bad problem), ENOMEM, EDEVICE. */
GRMHD_API int grmhd_init(const grmhd_problem *p, void *hip_stream, grmhd_ctx **out);

/* Device memory a context for problem p would own (geometry tables and
 * scratch: ctx_bytes) and the size of one caller-owned state (state_bytes),
 * without touching a device; for admission under a memory budget.
 * Errors: EINVAL (bad problem or NULL argument). */
GRMHD_API int grmhd_context_bytes(const grmhd_problem *p, int64_t *ctx_bytes, int64_t *state_bytes);

/* Release everything the context owns. NULL is accepted. */
GRMHD_API int grmhd_free(grmhd_ctx *ctx);

/* shape = {8, n3+6, n2+6, n1p}, strides in elements, and the element offset
 * of interior zone (0,0,0) of variable 0. */
GRMHD_API int grmhd_state_layout(const grmhd_ctx *ctx, int64_t shape[4], int64_t strides[4],
                       int64_t *interior_offset);

/* Conserved variables of the interior zones of P (ghosts of U are not
 * written). Functionality / Implementation Notes: U(P) is the analytic map. */
GRMHD_API int grmhd_prim_to_cons(grmhd_ctx *ctx, const double *P, double *U);

/* 1D_W inversion of the interior zones (Implementation Notes). P is the
 * Newton guess on entry and the result on exit. opts: GRMHD_OPT_FLOORS applies
 * the bounds (if the problem has floors), GRMHD_OPT_FIXUP repairs failed zones
 * from their neighbours. flags (nullable, same zone layout as one variable of
 * a state, int8): 1 where the inversion failed, 0 elsewhere (interior only).
 * n_fail (nullable, host): number of failed zones; synchronises. */
GRMHD_API int grmhd_cons_to_prim(grmhd_ctx *ctx, const double *U, double *P, int8_t *flags,
                       int32_t opts, int64_t *n_fail);

/* Courant step of state P: dt = cfl / sum_d (max_faces ctop_d / dx_d) with
 * ctop the LLF signal speed at each face. Refills the ghost zones of P.
 * dt (host) is written; synchronises. */
GRMHD_API int grmhd_get_dt(grmhd_ctx *ctx, double *P, double *dt);

/* One second-order predictor-corrector step of size dt, in place on P
 * (ghosts refilled). dt_next (nullable, host): the Courant step from the
 * corrector's signal speeds. Synchronises (it reads the step's counters back).
 * Returns GRMHD_ESTATE, whether or not dt_next is given, if the step stored a
 * non-finite value anywhere in P (a failed inversion that the fixup repairs
 * does not count) or a corrector signal speed is not finite. */
GRMHD_API int grmhd_step(grmhd_ctx *ctx, double *P, double dt, double *dt_next);

/* nsteps predictor-corrector steps in place on P with the step size kept on
 * the device: step n+1 uses min(cfl / sum_d (ctop_d / dx_d), 1.3 dt_n) from
 * step n's corrector speeds, the same rule, evaluated in the same order, as a
 * host loop of dt <- min(dt_next, 1.3 dt) around grmhd_step, so the results
 * are identical; the host does not wait between steps. dt (host, in/out): the
 * first step's size on entry, the size for the step after the last on exit.
 * Synchronises once at the end. Returns GRMHD_ESTATE if a step stored a
 * non-finite value in P or met a non-finite signal speed (dt then stops
 * growing). */
GRMHD_API int grmhd_run(grmhd_ctx *ctx, double *P, int32_t nsteps, double *dt);

/* The pieces of a step, for drivers that own the ghost zones of some
 * boundaries themselves (a domain split over several contexts exchanging
 * halos). grmhd_step(ctx, P, dt) is: fill_ghosts(P, P); substep(P, P, P_h,
 * dt/2, 0); fill_ghosts(P_h, P); substep(P_h, P, P, dt, 1).
 *
 * grmhd_fill_ghosts: the ghost zones of P from the problem's boundary
 * conditions, x1 then x2 then x3; DIRICHLET ghosts are copied from base (NULL:
 * P's own are kept). Asynchronous.
 * grmhd_substep: one predictor or corrector substep without the ghost fill:
 * P_out = bounds(invert(U(P_b) + dt L(P_s))) then the fixup, with L from P_s's
 * face fluxes (its ghost zones must be valid) and the geometric source at P_s.
 * P_out may be P_b. want_speeds != 0 records the per-direction maximum signal
 * speeds of this substep's faces with an interior transverse index.
 * Asynchronous.
 * grmhd_speeds: those three maxima (ctop_1, ctop_2, ctop_3), host array;
 * synchronises; GRMHD_ESTATE if one is not finite. */
GRMHD_API int grmhd_fill_ghosts(grmhd_ctx *ctx, double *P, const double *base);
GRMHD_API int grmhd_substep(grmhd_ctx *ctx, const double *Ps, const double *Pb, double *Pout, double dt,
                            int32_t want_speeds);
GRMHD_API int grmhd_speeds(grmhd_ctx *ctx, double ctop[3]);
/* grmhd_substep in two halves, for a split domain whose parts must exchange
 * the new state and the failure flags of their boundary planes before the
 * fixup (so that a failed zone next to a part boundary is repaired from the
 * same neighbours as in the undivided domain).
 *
 * grmhd_update: the substep without the fixup; P_out holds the bounded
 * inversion (a failed zone keeps the flux state's hydro primitives) and flags
 * (caller-owned int8 device array with the layout of one state variable,
 * [n3+6][n2+6][n1p]) is set to 1 on failed interior zones and 0 on the others
 * (its ghost cells are not written). Asynchronous.
 * grmhd_fixup: repairs every flagged interior zone of P, after grmhd_update on
 * the same context, from the mean of the hydro primitives of its non-flagged
 * neighbours among the 26 (the values grmhd_update stored, whatever the order),
 * then applies the bounds to it. Across a periodic direction the neighbours
 * are the zones on the other side of the seam; across a side whose bit is set
 * in halo_sides (bit 2 d + s for direction d = 0, 1, 2 and side s = 0 lower,
 * 1 upper) they are the first ghost layer of P and flags, which the caller has
 * filled with the neighbouring part's values and flags; across any other edge
 * there are none. grmhd_substep(..., Pout, ...) is grmhd_update followed by
 * grmhd_fixup with the context's own flags and no halo sides. Asynchronous.
 * Errors: EINVAL (NULL, dt, a halo side on a periodic direction). */
GRMHD_API int grmhd_update(grmhd_ctx *ctx, const double *Ps, const double *Pb, double *Pout, double dt,
                           int32_t want_speeds, int8_t *flags);
GRMHD_API int grmhd_fixup(grmhd_ctx *ctx, double *P, const int8_t *flags, int32_t halo_sides);
/* The Courant step of a domain split into nparts contexts: ctop (host,
 * nparts x 3) holds each part's grmhd_speeds; with c_d the maximum over the
 * parts, dt = cfl / sum_d (c_d / dx_d) (the rule grmhd_step uses for dt_next),
 * cfl and dx_d from ctx (any part: they share both). No device work.
 * Errors: EINVAL (NULL, nparts < 1, a negative speed), ESTATE (a non-finite
 * speed). */
GRMHD_API int grmhd_courant_dt(const grmhd_ctx *ctx, const double *ctop, int32_t nparts, double *dt);

/* ---- Electron heating (Implementation Notes: iharm3D tracks the dissipation
 * and splits it between ions and electrons after Ressler et al. 2015, with the
 * heating models of Howes 2010, Kawazura et al. 2019, Werner et al. 2018,
 * Rowan et al. 2017 and Sharma et al. 2007; with electron temperatures evolved, the bounds also keep
 * P_gas / rho^gamma below 3).
 *
 * E: caller-owned float64 device array [2][n3 + 6][n2 + 6][n1p], the state
 * layout with two variables (same strides as a state): the total entropy
 * K_tot = P_gas / rho^gam and the electron entropy K_e = P_e / rho^(4/3).
 *
 * grmhd_step_electrons: one predictor-corrector step as grmhd_step, in place
 * on P and E, in which every substep also
 *   - advects both entropies with the mass flux: sqrt(-g) rho u^t K is updated
 *     conservatively with face fluxes F_mass K*, K* the face value from the
 *     problem's reconstruction on the upwind side of F_mass;
 *   - after the other bounds and the fixup, lowers u to 3 rho^gam / (gam - 1)
 *     where it is above;
 *   - sets K_tot to the entropy of the new state and gives the electrons the
 *     fraction f_e of the heat the difference implies:
 *     K_e = K_e,adv + f_e (1/3)/(gam - 1) rho^(gam - 4/3) (K_tot - K_tot,adv),
 *     held within [0, rho^(gam - 4/3) K_tot] (0 <= P_e <= P_gas).
 * model: GRMHD_HEAT_CONSTANT (f_e = fel, 0 <= fel <= 1) or one of the five
 * models (fel ignored). The ghost zones of E follow the primitives' rules
 * without the axis sign change and the inflow fix. The first call on a context
 * allocates 4 doubles per padded zone of scratch, held until grmhd_free.
 * dt_next and the errors as grmhd_step (a non-finite entropy also gives
 * GRMHD_ESTATE); EINVAL also for an unknown model or fel outside [0, 1]. */
enum {
  GRMHD_HEAT_CONSTANT = 0, GRMHD_HEAT_KAWAZURA = 1, GRMHD_HEAT_WERNER = 2, GRMHD_HEAT_ROWAN = 3,
  GRMHD_HEAT_HOWES = 4, GRMHD_HEAT_SHARMA = 5
};
GRMHD_API int grmhd_step_electrons(grmhd_ctx *ctx, double *P, double *E, double dt, int32_t model, double fel,
                                   double *dt_next);
/* nsteps such steps with the step size kept on the device, as grmhd_run does
 * for grmhd_step (same rule, same results as a host loop of dt <- min(dt_next,
 * 1.3 dt) around grmhd_step_electrons). dt (host, in/out) as for grmhd_run;
 * errors as grmhd_run and grmhd_step_electrons. */
GRMHD_API int grmhd_run_electrons(grmhd_ctx *ctx, double *P, double *E, int32_t nsteps, double *dt, int32_t model,
                                  double fel);

/* max |div B| over cell corners, with div B the corner-centred divergence of
 * sqrt(-g) B (the quantity Flux-CT keeps at round-off, Implementation Notes).
 * Corners on non-periodic boundaries are excluded. Reads interior zones only.
 * max_divb (host) is written; synchronises. */
GRMHD_API int grmhd_divb(grmhd_ctx *ctx, const double *P, double *max_divb);

/* grmhd_divb for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same value as grmhd_divb, bit for bit, but its per-block partial maxima live
 * in a static device array of the library (65536 slots of 8 bytes plus the
 * result, 512 KiB, one copy per device, held until the process ends) instead
 * of the context's scratch; the call allocates nothing. Every call on a device
 * shares that device's array: calls that overlap on one device (several
 * streams or host threads) race and must be serialised by the caller. The
 * grid must need at most 65536 slots, ceil(n1/64) * ceil(n2/4) * n3 <= 65536
 * (the 288 x 128 x 128 torus needs 20480), else EINVAL. max_divb (host) is
 * written; synchronises. Errors: EINVAL, EDEVICE. */
GRMHD_API int grmhd_divb_noalloc(grmhd_ctx *ctx, const double *P, double *max_divb);

/* Failed-inversion count of the last step taken by grmhd_step or grmhd_run
 * (both substeps); synchronises. */
GRMHD_API int grmhd_step_failures(grmhd_ctx *ctx, int64_t *n_fail);

/* Kernel timing for measurement. grmhd_profile(ctx, 1) clears the record and
 * starts bracketing every kernel launch of grmhd_step, grmhd_run and the
 * electron calls (GRMHD_K_ELECTRONS: the scalar ghosts, advection and
 * heating) of the classes chosen with grmhd_profile_kernels (default: all)
 * with HIP events on the context stream; grmhd_profile(ctx, 0) stops. grmhd_profile_read returns, for
 * one kernel class, the summed device time in ms and the launch count since
 * the last clear; synchronises. Timing adds two event records per launch.
 * GRMHD_K_SWEEPS is the face-flux pass of all three directions, one launch per
 * substep. */
enum {
  GRMHD_K_GHOSTS = 0, GRMHD_K_SWEEPS = 1, /* 2, 3: unused (no launches) */
  GRMHD_K_UPDATE = 4, GRMHD_K_FIXUP = 5, GRMHD_K_ELECTRONS = 6, GRMHD_K_COUNT = 7
};
GRMHD_API int grmhd_profile(grmhd_ctx *ctx, int32_t enable);
/* Which kernel classes grmhd_profile brackets: mask is a set of bits
 * (1 << GRMHD_K_*); the launches of the other classes run without events (each
 * event record costs the stream a few microseconds, so a measurement that
 * needs only some classes times those alone). Default: every class. Takes
 * effect for launches enqueued after the call; the record is not cleared.
 * Errors: EINVAL (null context, empty mask or a bit outside the classes). */
GRMHD_API int grmhd_profile_kernels(grmhd_ctx *ctx, int32_t mask);
GRMHD_API int grmhd_profile_read(grmhd_ctx *ctx, int32_t kernel, double *total_ms, int64_t *launches);

/* Thread-block tile of the face-flux kernel (GRMHD_TILE_SWEEP) or of the
 * update and fixup kernels (GRMHD_TILE_UPDATE): tx zones along x1 by ty along
 * x2, one thread per zone (the face-flux kernel computes up to the three
 * lower faces of its zone); tx a power of two in [16, 256], tx * ty a multiple
 * of 64 and at most 512 (sweeps) or 256 (update). Defaults: sweeps 64 x 8,
 * update 64 x 1. Results do not depend on the tile. A batch uses the tiles of
 * its first job for every job. Errors: EINVAL. */
enum { GRMHD_TILE_SWEEP = 0, GRMHD_TILE_UPDATE = 1 };
GRMHD_API int grmhd_set_tiles(grmhd_ctx *ctx, int32_t which, int32_t tx, int32_t ty);
GRMHD_API int grmhd_get_tiles(const grmhd_ctx *ctx, int32_t which, int32_t *tx, int32_t *ty);

/* ---- Many independent problems advanced together.
 *
 * A batch groups n contexts (created with grmhd_init on the same device; all
 * with the same recon and precision) and advances every active one with one
 * grid per kernel phase spanning all of them, so small and uneven grids fill
 * the device together. One step of all active jobs is captured once into a
 * HIP graph and replayed. Each job keeps its own time step on the device:
 * after every step dt_j <- min(cfl / sum_d(ctop_d/dx_d), 1.3 dt_j) from its own
 * corrector signal speeds, so a job's evolution does not depend on the other
 * jobs in the batch. Each job uses its context's scratch; a context must not
 * be stepped on its own while it belongs to a live batch.
 * hip_stream: the stream everything is enqueued on; NULL makes the batch
 * create its own (graphs cannot be captured on the null stream). */
typedef struct grmhd_batch grmhd_batch;
GRMHD_API int grmhd_batch_create(grmhd_ctx *const *jobs, int32_t n, void *hip_stream, grmhd_batch **out);
/* Set the step size of every job (host array of n); asynchronous. */
GRMHD_API int grmhd_batch_set_dt(grmhd_batch *b, const double *dt);
/* Read every job's current step size and status (host arrays of n, either
 * nullable); status is 1 for a job whose signal speeds became non-finite;
 * synchronises. */
GRMHD_API int grmhd_batch_get(grmhd_batch *b, double *dt, int32_t *status);
/* nsteps steps of every job j with active[j] != 0 (active NULL: all) on state
 * P[j] (layout of job j's context, ghosts refilled). When P or active differ
 * from the previous call the job table is re-uploaded and the step graph
 * re-captured (synchronises once); otherwise asynchronous. */
GRMHD_API int grmhd_batch_step(grmhd_batch *b, double *const *P, const int32_t *active, int32_t nsteps);
/* As grmhd_batch_step, with electron heating (as grmhd_step_electrons) for
 * every active job j with E[j] != NULL, with its own heating model model[j]
 * and constant fraction fel[j] (host arrays of n; entries of jobs without
 * entropies are ignored). A job's evolution (P and E) is the same as a loop of
 * grmhd_step_electrons (or grmhd_step, without E) on its own context with
 * dt <- min(dt_next, 1.3 dt). The first call with entropies for a context
 * allocates its electron scratch. A change of any E[j], model[j] or fel[j]
 * re-captures the step graph. Errors: as grmhd_batch_step; EINVAL for an
 * unknown model or fel outside [0, 1]; ENOMEM. */
GRMHD_API int grmhd_batch_step_electrons(grmhd_batch *b, double *const *P, double *const *E, const int32_t *model,
                                         const double *fel, const int32_t *active, int32_t nsteps);
/* Kernel timing of batch steps, as grmhd_profile / grmhd_profile_read for a
 * context (same kernel classes, each launch spanning every active job). While
 * profiling is on, grmhd_batch_step enqueues its launches directly, each
 * bracketed by two events, instead of replaying the captured graph: the same
 * kernels in the same order, so results are unchanged. */
GRMHD_API int grmhd_batch_profile(grmhd_batch *b, int32_t enable);
GRMHD_API int grmhd_batch_profile_read(grmhd_batch *b, int32_t kernel, double *total_ms, int64_t *launches);
GRMHD_API int grmhd_batch_free(grmhd_batch *b);
GRMHD_API const char *grmhd_batch_last_error(const grmhd_batch *b);

GRMHD_API const char *grmhd_strerror(int status);
GRMHD_API const char *grmhd_last_error(const grmhd_ctx *ctx);
GRMHD_API int grmhd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GRMHD_H */
