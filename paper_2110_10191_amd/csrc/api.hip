// Host side of the C ABI declared in grmhd.h: validation, context lifetime,
// geometry set-up, and the sequencing of kernels for each call.
//
// One step (second-order predictor-corrector, HARM scheme):
//   predictor: ghosts(P); sweeps(P); update(F, P_base = P, P_s = P, dt/2) -> P_h; fixup
//   corrector: ghosts(P_h); sweeps(P_h) + ctop; update(F, P, P_h, dt) -> P; fixup
// Everything is enqueued on the context's stream; nothing waits on the host
// unless a host scalar is requested.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

namespace {

thread_local std::string g_init_error;

int fail(grmhd_ctx* c, int status, const std::string& msg) {
  if (c) c->err = msg;
  else g_init_error = msg;
  return status;
}

int hip_fail(grmhd_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, GRMHD_EDEVICE, m);
}

#define HIP_OR_FAIL(ctx, call, where)            \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
  } while (0)

int validate(const grmhd_problem* p, std::string& why) {
  if (!p) { why = "problem is NULL"; return GRMHD_EINVAL; }
  if (p->n1 < 1 || p->n2 < 1 || p->n3 < 1) { why = "n1, n2, n3 must be >= 1"; return GRMHD_EINVAL; }
  if (p->coords < GRMHD_MINKOWSKI_CART || p->coords > GRMHD_KERR_CKS) { why = "unknown coords"; return GRMHD_EINVAL; }
  if (p->recon != GRMHD_RECON_MC && p->recon != GRMHD_RECON_WENO5) { why = "unknown recon"; return GRMHD_EINVAL; }
  if (p->precision != GRMHD_FP64 && p->precision != GRMHD_MIXED) { why = "unknown precision"; return GRMHD_EINVAL; }
  if (!(p->gam > 1.0) || !(p->cfl > 0.0) || !std::isfinite(p->gam) || !std::isfinite(p->cfl)) {
    why = "need gam > 1 and cfl > 0";
    return GRMHD_EINVAL;
  }
  const double lo[3] = {p->x1min, p->x2min, p->x3min}, hi[3] = {p->x1max, p->x2max, p->x3max};
  const int n[3] = {p->n1, p->n2, p->n3};
  for (int d = 0; d < 3; ++d) {
    if (!(hi[d] > lo[d]) || !std::isfinite(lo[d]) || !std::isfinite(hi[d])) {
      why = "each extent needs xmax > xmin";
      return GRMHD_EINVAL;
    }
    for (int s = 0; s < 2; ++s)
      if (p->bc[d][s] < GRMHD_BC_PERIODIC || p->bc[d][s] > GRMHD_BC_DIRICHLET) {
        why = "unknown boundary type";
        return GRMHD_EINVAL;
      }
    const bool per0 = p->bc[d][0] == GRMHD_BC_PERIODIC, per1 = p->bc[d][1] == GRMHD_BC_PERIODIC;
    if (per0 != per1) { why = "periodic boundaries must be periodic on both sides"; return GRMHD_EINVAL; }
    if (!per0 && n[d] < NG) { why = "non-periodic directions need at least 3 zones"; return GRMHD_EINVAL; }
    for (int s = 0; s < 2; ++s) {
      if (p->bc[d][s] == GRMHD_BC_OUTFLOW && d != 0) { why = "outflow boundaries are x1 only"; return GRMHD_EINVAL; }
      if (p->bc[d][s] == GRMHD_BC_POLAR && d != 1) { why = "polar boundaries are x2 only"; return GRMHD_EINVAL; }
    }
  }
  if (p->coords == GRMHD_MINKOWSKI_CART) {
    if (p->floors) { why = "floors need a Kerr metric (they depend on r)"; return GRMHD_EINVAL; }
    if (p->bc[0][0] == GRMHD_BC_OUTFLOW || p->bc[0][1] == GRMHD_BC_OUTFLOW) {
      why = "outflow boundaries need a Kerr metric";
      return GRMHD_EINVAL;
    }
  } else {
    if (!(std::fabs(p->a) < 1.0)) { why = "need |a| < 1"; return GRMHD_EINVAL; }
    if (p->coords == GRMHD_KERR_FMKS && !(p->poly_xt > 0.0)) { why = "need poly_xt > 0"; return GRMHD_EINVAL; }
  }
  if (p->coords == GRMHD_KERR_CKS) {
    for (int d = 0; d < 3; ++d)
      for (int s = 0; s < 2; ++s)
        if (p->bc[d][s] != GRMHD_BC_PERIODIC && p->bc[d][s] != GRMHD_BC_DIRICHLET) {
          why = "Cartesian Kerr-Schild boundaries are periodic or Dirichlet";
          return GRMHD_EINVAL;
        }
    // the point of the padded box nearest the origin must have R >= 1 (then r > 0)
    double r2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double pad = NG * (hi[d] - lo[d]) / n[d];
      const double a = lo[d] - pad, b = hi[d] + pad;
      const double q = a > 0.0 ? a : (b < 0.0 ? -b : 0.0);
      r2 += q * q;
    }
    if (!(r2 >= 1.0)) { why = "the Cartesian Kerr-Schild box (ghosts included) must lie outside the unit sphere"; return GRMHD_EINVAL; }
  }
  if (p->floors && !(p->sigma_max > 0 && p->uorho_max > 0 && p->gamma_max > 1.0 && p->beta_min >= 0)) {
    why = "bad floor parameters";
    return GRMHD_EINVAL;
  }
  const long long p1 = ((p->n1 + 2 * NG + 7) / 8) * 8;
  const long long cells = p1 * (p->n2 + 2 * NG) * (long long)(p->n3 + 2 * NG);
  if (cells * NV >= (1ll << 31)) { why = "grid too large for 32-bit indexing of one state"; return GRMHD_EINVAL; }
  if (p->coords == GRMHD_KERR_CKS && cells * N_CENT >= (1ll << 31)) {
    why = "grid too large for 32-bit indexing of the 3D geometry tables (at most 2^25 padded zones)";
    return GRMHD_EINVAL;
  }
  return GRMHD_OK;
}

Dims make_dims(const grmhd_problem& p) {
  Dims d;
  d.n1 = p.n1;
  d.n2 = p.n2;
  d.n3 = p.n3;
  d.p1 = ((p.n1 + 2 * NG + 7) / 8) * 8;
  d.p2 = p.n2 + 2 * NG;
  d.p3 = p.n3 + 2 * NG;
  d.s2 = d.p1;
  d.s3 = d.p2 * d.p1;
  d.sv = d.p3 * d.s3;
  const bool k3 = p.coords == GRMHD_KERR_CKS;
  d.ts = k3 ? d.sv : d.p2 * d.p1;
  d.tk = k3 ? d.s3 : 0;
  d.stx = SWEEP_TILE_X;
  d.utx = TILE_X;
  d.sty = SWEEP_TILE_Y;
  d.uty = TILE_Y;
  d.out_lo = p.bc[0][0] == GRMHD_BC_OUTFLOW;
  d.out_hi = p.bc[0][1] == GRMHD_BC_OUTFLOW;
  return d;
}

void free_all(grmhd_ctx* c) {
  void* ptrs[] = {c->t.cent, c->t.f1, c->t.f2, c->t.f3, c->t.f1f, c->t.f2f, c->t.f3f,
                  c->Ph, c->F[0], c->F[1], c->F[2], c->flags, c->ctr, c->Eh, c->Uk};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
}

template <typename T>
hipError_t dalloc(T** ptr, size_t bytes) {
  return hipMalloc((void**)ptr, bytes);
}


// the electron entropies of a substep: flux state Es (ghosts refilled here),
// base state Eb (also the source of Dirichlet ghosts), result Eout
struct ElectronPass {
  double* Es;
  const double* Eb;
  double* Eout;
  int model;
  double fel;
};

// predictor or corrector substep; Pb is the base state (also the source of
// Dirichlet ghosts). dt_dev: when not null the step is dt_scale * *dt_dev (read
// on the device). fill = false leaves the ghost zones of Ps as they are.
// el: also advect and heat the electron entropies.
// flags: the failure flags the update writes (the context's own when null);
// fix: run the fixup (with the context's flags and no halo sides) as well.
// extra_reset: further counters to clear first (8: the step's totals);
// dtr: first set the device step size from the previous step's counters.
int substep(grmhd_ctx* c, double* Ps, double* Pb, double* Pout, double dt, bool want_ctop,
            const double* dt_dev = nullptr, double dt_scale = 1.0, bool fill = true,
            const ElectronPass* el = nullptr, int8_t* flags = nullptr, bool fix = true, int extra_reset = 0,
            const DtRule* dtr = nullptr) {
  int8_t* fl = flags ? flags : c->flags;
  hipStream_t s = c->stream;
  // the counters the face fluxes and the update count into start at zero (the
  // ghost fill clears them when there is one)
  const int reset_mask = (want_ctop ? (1 | 4) : 4) | extra_reset;
  if (fill) {
    ProfScope ps(c->prof, s, GRMHD_K_GHOSTS);
    HIP_OR_FAIL(c, launch_fill_ghosts(c->p, c->d, c->t, Ps, Pb, s, c->ctr, reset_mask, dtr ? *dtr : DtRule{}),
                "ghost fill");
  } else {
    if (dtr) HIP_OR_FAIL(c, launch_ctx_dt(c->ctr, dtr->cfl, dtr->dx[0], dtr->dx[1], dtr->dx[2], s), "dt");
    HIP_OR_FAIL(c, launch_reset(c->ctr, reset_mask, s), "reset");
  }
  if (el) {
    ProfScope ps(c->prof, s, GRMHD_K_ELECTRONS);
    HIP_OR_FAIL(c, launch_fill_scalar_ghosts(c->p, c->d, el->Es, el->Eb, s), "scalar ghost fill");
  }
  {
    ProfScope ps(c->prof, s, GRMHD_K_SWEEPS);
    HIP_OR_FAIL(c, launch_sweeps(c->p, c->mixed, c->d, c->t, Ps, c->F, want_ctop ? c->ctr->ctop : nullptr,
                                 s),
                "sweeps");
  }
  if (el) {
    // before the update: in the corrector it overwrites the base state in place
    ProfScope ps(c->prof, s, GRMHD_K_ELECTRONS);
    HIP_OR_FAIL(c, launch_scalar_advect(c->mixed, c->p.recon, c->d, c->t, c->up, c->F[0], c->F[1], c->F[2], Pb,
                                        el->Eb, el->Es, c->Uk, dt, dt_dev, dt_scale, s),
                "scalar advection");
  }
  {
    ProfScope ps(c->prof, s, GRMHD_K_UPDATE);
    HIP_OR_FAIL(c, launch_update(c->mixed, c->d, c->t, c->up, c->F[0], c->F[1], c->F[2], Pb, Ps, Pout,
                                 fl, dt, dt_dev, dt_scale, c->ctr, s,
                                 c->p.coords == GRMHD_KERR_CKS ? &c->p : nullptr),
                "update");
  }
  if (fix) {
    ProfScope ps(c->prof, s, GRMHD_K_FIXUP);
    HIP_OR_FAIL(c, launch_fixup(c->d, c->t, c->up, Pout, fl, c->ctr, 0, s), "fixup");
  }
  if (el) {
    ProfScope ps(c->prof, s, GRMHD_K_ELECTRONS);
    HIP_OR_FAIL(c, launch_electron_heat(c->d, c->t, c->p.gam, Pout, c->Uk, el->Eout, el->model, el->fel, c->ctr, s),
                "electron heating");
  }
  return GRMHD_OK;
}

// the context's counters on the host; synchronises
int read_counters(grmhd_ctx* c, Counters* h) {
  HIP_OR_FAIL(c, hipMemcpyAsync(h, c->ctr, sizeof(Counters), hipMemcpyDeviceToHost, c->stream), "copy counters");
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream), "synchronize");
  return GRMHD_OK;
}

int read_speeds(grmhd_ctx* c, double v[3]) {
  Counters h;
  const int st = read_counters(c, &h);
  if (st != GRMHD_OK) return st;
  for (int d = 0; d < 3; ++d) std::memcpy(&v[d], &h.ctop[d], sizeof(double));
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(v[d])) return fail(c, GRMHD_ESTATE, "non-finite signal speed in the state");
  return GRMHD_OK;
}

// dt = cfl / sum_d (ctop_d / dx_d): the Courant rule of the method, on the host
double courant_dt(double cfl, const double ctop[3], const double dx[3]) {
  double sum = 0.0;
  for (int d = 0; d < 3; ++d) sum += ctop[d] / dx[d];
  return sum > 0.0 ? cfl / sum : INFINITY;
}

int read_dt(grmhd_ctx* c, double* dt) {
  double v[3];
  const int st = read_speeds(c, v);
  if (st != GRMHD_OK) return st;
  *dt = courant_dt(c->p.cfl, v, c->dx);
  return GRMHD_OK;
}

// after a step: GRMHD_ESTATE if a non-finite value was stored in the state or
// a corrector signal speed is not finite; dt_next (nullable) from the speeds
int finish_step(grmhd_ctx* c, double* dt_next) {
  Counters h;
  const int st = read_counters(c, &h);
  if (st != GRMHD_OK) return st;
  if (h.bad) return fail(c, GRMHD_ESTATE, "non-finite value in the state after the step");
  double v[3];
  for (int d = 0; d < 3; ++d) std::memcpy(&v[d], &h.ctop[d], sizeof(double));
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(v[d])) return fail(c, GRMHD_ESTATE, "non-finite signal speed in the state");
  if (dt_next) *dt_next = courant_dt(c->p.cfl, v, c->dx);
  return GRMHD_OK;
}

// argument checks of the electron calls, and their scratch on first use
int electron_prep(grmhd_ctx* ctx, const double* P, const double* E, int32_t model, double fel, const char* who) {
  std::string w(who);
  if (!P || !E) return fail(ctx, GRMHD_EINVAL, w + ": NULL state");
  if (!heat_args_ok(model, fel)) return fail(ctx, GRMHD_EINVAL, w + ": unknown heating model or fel outside [0, 1]");
  const hipError_t e = ctx_electron_scratch(ctx);
  if (e == hipErrorOutOfMemory) return fail(ctx, GRMHD_ENOMEM, w + ": scratch allocation failed");
  HIP_OR_FAIL(ctx, e, "electron scratch");
  return GRMHD_OK;
}

// nsteps steps with the step size kept on the device (E, model, fel: with
// electron heating when E is not null)
int run_steps(grmhd_ctx* ctx, double* P, double* E, int32_t model, double fel, int32_t nsteps, double* dt) {
  struct {
    double dt;
    int status;
  } host{*dt, 0};
  HIP_OR_FAIL(ctx, hipMemcpyAsync(&ctx->ctr->dt, &host.dt, sizeof(double), hipMemcpyHostToDevice, ctx->stream),
              "set dt");
  HIP_OR_FAIL(ctx, hipMemcpyAsync(&ctx->ctr->status, &host.status, sizeof(int), hipMemcpyHostToDevice, ctx->stream),
              "set status");
  const double* dtp = &ctx->ctr->dt;
  const ElectronPass pred{E, E, ctx->Eh, model, fel};
  const ElectronPass corr{ctx->Eh, E, E, model, fel};
  // each step's predictor ghost fill first takes the step size from the
  // previous step's counters (the host's dt for the first step), then clears
  // the step's totals; the last step's rule runs after the loop
  const DtRule rule{1, ctx->p.cfl, {ctx->dx[0], ctx->dx[1], ctx->dx[2]}};
  for (int s = 0; s < nsteps; ++s) {
    int st = substep(ctx, P, P, ctx->Ph, 0.0, false, dtp, 0.5, true, E ? &pred : nullptr, nullptr, true, 8,
                     s > 0 ? &rule : nullptr);
    if (st != GRMHD_OK) return st;
    st = substep(ctx, ctx->Ph, P, P, 0.0, true, dtp, 1.0, true, E ? &corr : nullptr);
    if (st != GRMHD_OK) return st;
  }
  if (nsteps > 0)
    HIP_OR_FAIL(ctx, launch_ctx_dt(ctx->ctr, ctx->p.cfl, ctx->dx[0], ctx->dx[1], ctx->dx[2], ctx->stream), "dt");
  HIP_OR_FAIL(ctx, hipMemcpyAsync(&host.dt, &ctx->ctr->dt, sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
              "read dt");
  HIP_OR_FAIL(ctx, hipMemcpyAsync(&host.status, &ctx->ctr->status, sizeof(int), hipMemcpyDeviceToHost, ctx->stream),
              "read status");
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
  *dt = host.dt;
  if (host.status) return fail(ctx, GRMHD_ESTATE, "non-finite signal speed or state value");
  return GRMHD_OK;
}

}  // namespace

bool heat_args_ok(int32_t model, double fel) {
  if (model < GRMHD_HEAT_CONSTANT || model > GRMHD_HEAT_SHARMA) return false;
  return model != GRMHD_HEAT_CONSTANT || (fel >= 0.0 && fel <= 1.0);
}

hipError_t ctx_electron_scratch(grmhd_ctx* c) {
  if (c->Eh) return hipSuccess;
  const size_t bytes = (size_t)GRMHD_NSCALAR * c->d.sv * sizeof(double);
  hipError_t e = hipMalloc((void**)&c->Eh, bytes);
  if (e == hipSuccess) e = hipMalloc((void**)&c->Uk, bytes);
  // ghost and padding zones of the half-step entropies that no rule writes stay finite
  if (e == hipSuccess) e = hipMemsetAsync(c->Eh, 0, bytes, c->stream);
  if (e != hipSuccess) {
    if (c->Eh) (void)hipFree(c->Eh);
    if (c->Uk) (void)hipFree(c->Uk);
    c->Eh = c->Uk = nullptr;
  }
  return e;
}

extern "C" {

int grmhd_version(void) { return 1; }

const char* grmhd_strerror(int status) {
  switch (status) {
    case GRMHD_OK: return "ok";
    case GRMHD_EINVAL: return "invalid argument";
    case GRMHD_ENOMEM: return "out of device memory";
    case GRMHD_EDEVICE: return "device or runtime error";
    case GRMHD_EUNSUPPORTED: return "unsupported";
    case GRMHD_ESTATE: return "non-finite state";
    default: return "unknown status";
  }
}

const char* grmhd_last_error(const grmhd_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

int grmhd_context_bytes(const grmhd_problem* p, int64_t* ctx_bytes, int64_t* state_bytes) {
  if (!p || !ctx_bytes || !state_bytes) return fail(nullptr, GRMHD_EINVAL, "context_bytes: NULL argument");
  std::string why;
  const int st = validate(p, why);
  if (st != GRMHD_OK) return fail(nullptr, st, why);
  const Dims d = make_dims(*p);
  const size_t ts = (size_t)d.ts, sv = (size_t)d.sv;
  const size_t fsz = p->precision == GRMHD_MIXED ? sizeof(float) : sizeof(double);
  const size_t tables = (N_CENT + 3 * N_FACE) * ts * sizeof(double) + 3 * N_FACE * ts * sizeof(float);
  const size_t scratch = NV * sv * sizeof(double) + 3 * NV * sv * fsz + sv + sizeof(Counters);
  *ctx_bytes = (int64_t)(tables + scratch);
  *state_bytes = (int64_t)(NV * sv * sizeof(double));
  return GRMHD_OK;
}

int grmhd_init(const grmhd_problem* p, void* hip_stream, grmhd_ctx** out) {
  if (!out) return fail(nullptr, GRMHD_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  int st = validate(p, why);
  if (st != GRMHD_OK) return fail(nullptr, st, why);
  int ndev = 0;
  const hipError_t de = hipGetDeviceCount(&ndev);
  if (de != hipSuccess || ndev < 1)
    return fail(nullptr, GRMHD_EDEVICE,
                std::string("no HIP device (hipGetDeviceCount: ") + hipGetErrorString(de) + ")");

  grmhd_ctx* c = new grmhd_ctx();
  c->p = *p;
  c->d = make_dims(*p);
  c->stream = (hipStream_t)hip_stream;
  c->mixed = p->precision == GRMHD_MIXED;
  (void)hipGetDevice(&c->device);
  {
    const hipError_t se = noalloc_scratch(c->device, &c->noalloc);
    if (se != hipSuccess) {
      delete c;
      return fail(nullptr, GRMHD_EDEVICE, std::string("static scratch address: ") + hipGetErrorString(se));
    }
  }
  c->dx[0] = (p->x1max - p->x1min) / p->n1;
  c->dx[1] = (p->x2max - p->x2min) / p->n2;
  c->dx[2] = (p->x3max - p->x3min) / p->n3;
  c->up.gam = p->gam;
  c->up.sigma_max = p->sigma_max;
  c->up.beta_min = p->beta_min;
  c->up.uorho_max = p->uorho_max;
  c->up.gamma_max = p->gamma_max;
  c->up.dx1 = c->dx[0];
  c->up.dx2 = c->dx[1];
  c->up.dx3 = c->dx[2];
  c->up.idx1 = 1.0 / c->dx[0];
  c->up.idx2 = 1.0 / c->dx[1];
  c->up.idx3 = 1.0 / c->dx[2];
  c->up.floors = p->floors ? 1 : 0;
  c->up.polar_lo = p->bc[1][0] == GRMHD_BC_POLAR;
  c->up.polar_hi = p->bc[1][1] == GRMHD_BC_POLAR;
  for (int d = 0; d < 3; ++d) c->up.periodic[d] = p->bc[d][0] == GRMHD_BC_PERIODIC;

  const size_t ts = (size_t)c->d.ts, sv = (size_t)c->d.sv;
  const size_t fsz = c->mixed ? sizeof(float) : sizeof(double);
  // keep in step with context_bytes()
  bool ok = dalloc(&c->t.cent, N_CENT * ts * sizeof(double)) == hipSuccess &&
            dalloc(&c->t.f1, N_FACE * ts * sizeof(double)) == hipSuccess &&
            dalloc(&c->t.f2, N_FACE * ts * sizeof(double)) == hipSuccess &&
            dalloc(&c->t.f3, N_FACE * ts * sizeof(double)) == hipSuccess &&
            dalloc(&c->t.f1f, N_FACE * ts * sizeof(float)) == hipSuccess &&
            dalloc(&c->t.f2f, N_FACE * ts * sizeof(float)) == hipSuccess &&
            dalloc(&c->t.f3f, N_FACE * ts * sizeof(float)) == hipSuccess &&
            dalloc(&c->Ph, NV * sv * sizeof(double)) == hipSuccess &&
            dalloc(&c->F[0], NV * sv * fsz) == hipSuccess && dalloc(&c->F[1], NV * sv * fsz) == hipSuccess &&
            dalloc(&c->F[2], NV * sv * fsz) == hipSuccess && dalloc(&c->flags, sv) == hipSuccess &&
            dalloc(&c->ctr, sizeof(Counters)) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    free_all(c);
    delete c;
    return fail(nullptr, GRMHD_ENOMEM, "device allocation failed");
  }
  // one-time clears (outside any captured work); padding stays finite
  hipError_t e = hipMemsetAsync(c->t.cent, 0, N_CENT * ts * sizeof(double), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->Ph, 0, NV * sv * sizeof(double), c->stream);
  for (int q = 0; q < 3 && e == hipSuccess; ++q) e = hipMemsetAsync(c->F[q], 0, NV * sv * fsz, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->flags, 0, sv, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ctr, 0, sizeof(Counters), c->stream);
  if (e == hipSuccess) e = launch_geometry(c->p, c->d, c->t, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    std::string m = std::string("geometry set-up: ") + hipGetErrorString(e);
    free_all(c);
    delete c;
    return fail(nullptr, GRMHD_EDEVICE, m);
  }
  *out = c;
  return GRMHD_OK;
}

int grmhd_free(grmhd_ctx* ctx) {
  if (!ctx) return GRMHD_OK;
  (void)hipStreamSynchronize(ctx->stream);
  ctx->prof.destroy();
  free_all(ctx);
  delete ctx;
  return GRMHD_OK;
}

int grmhd_set_tiles(grmhd_ctx* ctx, int32_t which, int32_t tx, int32_t ty) {
  if (!ctx) return GRMHD_EINVAL;
  const bool pow2 = tx >= 16 && tx <= 256 && (tx & (tx - 1)) == 0;
  const int maxt = which == GRMHD_TILE_SWEEP ? SWEEP_MAX_THREADS : UPDATE_MAX_THREADS;
  if (!pow2 || ty < 1 || tx * ty > maxt || (tx * ty) % 64 != 0)
    return fail(ctx, GRMHD_EINVAL,
                "set_tiles: need tx a power of two in [16, 256], tx*ty a multiple of 64, at most 512 "
                "(sweeps) or 256 (update)");
  if (which == GRMHD_TILE_SWEEP) {
    ctx->d.stx = tx;
    ctx->d.sty = ty;
  } else if (which == GRMHD_TILE_UPDATE) {
    ctx->d.utx = tx;
    ctx->d.uty = ty;
  } else {
    return fail(ctx, GRMHD_EINVAL, "set_tiles: unknown kernel class");
  }
  return GRMHD_OK;
}

int grmhd_get_tiles(const grmhd_ctx* ctx, int32_t which, int32_t* tx, int32_t* ty) {
  if (!ctx || !tx || !ty) return GRMHD_EINVAL;
  if (which == GRMHD_TILE_SWEEP) {
    *tx = ctx->d.stx;
    *ty = ctx->d.sty;
  } else if (which == GRMHD_TILE_UPDATE) {
    *tx = ctx->d.utx;
    *ty = ctx->d.uty;
  } else {
    return GRMHD_EINVAL;
  }
  return GRMHD_OK;
}

int grmhd_profile(grmhd_ctx* ctx, int32_t enable) {
  if (!ctx) return GRMHD_EINVAL;
  if (enable) {
    HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    ctx->prof.clear();
  }
  ctx->prof.on = enable != 0;
  return GRMHD_OK;
}

int grmhd_profile_kernels(grmhd_ctx* ctx, int32_t mask) {
  if (!ctx) return GRMHD_EINVAL;
  if (mask <= 0 || (mask & ~((1 << GRMHD_K_COUNT) - 1)))
    return fail(ctx, GRMHD_EINVAL, "profile_kernels: mask must be a non-empty set of GRMHD_K_* bits");
  ctx->prof.mask = (unsigned)mask;
  return GRMHD_OK;
}

int grmhd_profile_read(grmhd_ctx* ctx, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches) return GRMHD_EINVAL;
  if (kernel < 0 || kernel >= GRMHD_K_COUNT) return fail(ctx, GRMHD_EINVAL, "profile_read: unknown kernel");
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
  HIP_OR_FAIL(ctx, ctx->prof.total(kernel, total_ms, launches), "event time");
  return GRMHD_OK;
}

int grmhd_state_layout(const grmhd_ctx* ctx, int64_t shape[4], int64_t strides[4], int64_t* interior_offset) {
  if (!ctx || !shape || !strides) return GRMHD_EINVAL;
  const Dims& d = ctx->d;
  shape[0] = NV;
  shape[1] = d.p3;
  shape[2] = d.p2;
  shape[3] = d.p1;
  strides[0] = d.sv;
  strides[1] = d.s3;
  strides[2] = d.s2;
  strides[3] = 1;
  if (interior_offset) *interior_offset = cell_of(d, 0, 0, 0);
  return GRMHD_OK;
}

int grmhd_prim_to_cons(grmhd_ctx* ctx, const double* P, double* U) {
  if (!ctx) return GRMHD_EINVAL;
  if (!P || !U) return fail(ctx, GRMHD_EINVAL, "prim_to_cons: NULL state");
  if (P == U) return fail(ctx, GRMHD_EINVAL, "prim_to_cons: P and U must differ");
  HIP_OR_FAIL(ctx, launch_prim_to_cons(ctx->d, ctx->t, ctx->p.gam, P, U, ctx->stream), "prim_to_cons");
  return GRMHD_OK;
}

int grmhd_cons_to_prim(grmhd_ctx* ctx, const double* U, double* P, int8_t* flags, int32_t opts, int64_t* n_fail) {
  if (!ctx) return GRMHD_EINVAL;
  if (!P || !U) return fail(ctx, GRMHD_EINVAL, "cons_to_prim: NULL state");
  if (P == U) return fail(ctx, GRMHD_EINVAL, "cons_to_prim: P and U must differ");
  if (opts & ~(GRMHD_OPT_FLOORS | GRMHD_OPT_FIXUP)) return fail(ctx, GRMHD_EINVAL, "cons_to_prim: unknown opts bits");
  UpdateParams up = ctx->up;
  up.floors = (ctx->p.floors && (opts & GRMHD_OPT_FLOORS)) ? 1 : 0;
  int8_t* fl = flags ? flags : ctx->flags;
  hipStream_t s = ctx->stream;
  HIP_OR_FAIL(ctx, launch_reset(ctx->ctr, 4, s), "reset");
  HIP_OR_FAIL(ctx, launch_cons_to_prim(ctx->d, ctx->t, up, U, P, fl, ctx->ctr, s), "cons_to_prim");
  if (opts & GRMHD_OPT_FIXUP) HIP_OR_FAIL(ctx, launch_fixup(ctx->d, ctx->t, up, P, fl, ctx->ctr, 0, s), "fixup");
  if (n_fail) {
    unsigned int nf = 0;
    HIP_OR_FAIL(ctx, hipMemcpyAsync(&nf, &ctx->ctr->fail, sizeof(nf), hipMemcpyDeviceToHost, s), "copy");
    HIP_OR_FAIL(ctx, hipStreamSynchronize(s), "synchronize");
    *n_fail = nf;
  }
  return GRMHD_OK;
}

int grmhd_get_dt(grmhd_ctx* ctx, double* P, double* dt) {
  if (!ctx) return GRMHD_EINVAL;
  if (!P || !dt) return fail(ctx, GRMHD_EINVAL, "get_dt: NULL argument");
  hipStream_t s = ctx->stream;
  HIP_OR_FAIL(ctx, launch_fill_ghosts(ctx->p, ctx->d, ctx->t, P, P, s), "ghost fill");
  HIP_OR_FAIL(ctx, launch_reset(ctx->ctr, 1, s), "reset");
  HIP_OR_FAIL(ctx, launch_sweeps(ctx->p, ctx->mixed, ctx->d, ctx->t, P, ctx->F, ctx->ctr->ctop, s),
              "sweeps");
  return read_dt(ctx, dt);
}

int grmhd_step(grmhd_ctx* ctx, double* P, double dt, double* dt_next) {
  if (!ctx) return GRMHD_EINVAL;
  if (!P) return fail(ctx, GRMHD_EINVAL, "step: NULL state");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, GRMHD_EINVAL, "step: dt must be finite and > 0");
  HIP_OR_FAIL(ctx, launch_reset(ctx->ctr, 8, ctx->stream), "reset");
  int st = substep(ctx, P, P, ctx->Ph, 0.5 * dt, false);
  if (st != GRMHD_OK) return st;
  st = substep(ctx, ctx->Ph, P, P, dt, true);
  if (st != GRMHD_OK) return st;
  return finish_step(ctx, dt_next);
}

int grmhd_step_electrons(grmhd_ctx* ctx, double* P, double* E, double dt, int32_t model, double fel,
                         double* dt_next) {
  if (!ctx) return GRMHD_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, GRMHD_EINVAL, "step_electrons: dt must be finite and > 0");
  int st = electron_prep(ctx, P, E, model, fel, "step_electrons");
  if (st != GRMHD_OK) return st;
  HIP_OR_FAIL(ctx, launch_reset(ctx->ctr, 8, ctx->stream), "reset");
  const ElectronPass pred{E, E, ctx->Eh, model, fel};
  st = substep(ctx, P, P, ctx->Ph, 0.5 * dt, false, nullptr, 1.0, true, &pred);
  if (st != GRMHD_OK) return st;
  const ElectronPass corr{ctx->Eh, E, E, model, fel};
  st = substep(ctx, ctx->Ph, P, P, dt, true, nullptr, 1.0, true, &corr);
  if (st != GRMHD_OK) return st;
  return finish_step(ctx, dt_next);
}

int grmhd_run(grmhd_ctx* ctx, double* P, int32_t nsteps, double* dt) {
  if (!ctx) return GRMHD_EINVAL;
  if (!P || !dt) return fail(ctx, GRMHD_EINVAL, "run: NULL argument");
  if (nsteps < 0) return fail(ctx, GRMHD_EINVAL, "run: nsteps < 0");
  if (!(*dt > 0.0) || !std::isfinite(*dt)) return fail(ctx, GRMHD_EINVAL, "run: dt must be finite and > 0");
  return run_steps(ctx, P, nullptr, 0, 0.0, nsteps, dt);
}

int grmhd_run_electrons(grmhd_ctx* ctx, double* P, double* E, int32_t nsteps, double* dt, int32_t model,
                        double fel) {
  if (!ctx) return GRMHD_EINVAL;
  if (!dt) return fail(ctx, GRMHD_EINVAL, "run_electrons: NULL argument");
  if (nsteps < 0) return fail(ctx, GRMHD_EINVAL, "run_electrons: nsteps < 0");
  if (!(*dt > 0.0) || !std::isfinite(*dt)) return fail(ctx, GRMHD_EINVAL, "run_electrons: dt must be finite and > 0");
  int st = electron_prep(ctx, P, E, model, fel, "run_electrons");
  if (st != GRMHD_OK) return st;
  return run_steps(ctx, P, E, model, fel, nsteps, dt);
}

int grmhd_fill_ghosts(grmhd_ctx* ctx, double* P, const double* base) {
  if (!ctx) return GRMHD_EINVAL;
  if (!P) return fail(ctx, GRMHD_EINVAL, "fill_ghosts: NULL state");
  HIP_OR_FAIL(ctx, launch_fill_ghosts(ctx->p, ctx->d, ctx->t, P, base ? base : P, ctx->stream), "ghost fill");
  return GRMHD_OK;
}

int grmhd_substep(grmhd_ctx* ctx, const double* Ps, const double* Pb, double* Pout, double dt, int32_t want_speeds) {
  if (!ctx) return GRMHD_EINVAL;
  if (!Ps || !Pb || !Pout) return fail(ctx, GRMHD_EINVAL, "substep: NULL state");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, GRMHD_EINVAL, "substep: dt must be finite and > 0");
  return substep(ctx, const_cast<double*>(Ps), const_cast<double*>(Pb), Pout, dt, want_speeds != 0, nullptr, 1.0,
                 false);
}

int grmhd_update(grmhd_ctx* ctx, const double* Ps, const double* Pb, double* Pout, double dt, int32_t want_speeds,
                 int8_t* flags) {
  if (!ctx) return GRMHD_EINVAL;
  if (!Ps || !Pb || !Pout || !flags) return fail(ctx, GRMHD_EINVAL, "update: NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(ctx, GRMHD_EINVAL, "update: dt must be finite and > 0");
  return substep(ctx, const_cast<double*>(Ps), const_cast<double*>(Pb), Pout, dt, want_speeds != 0, nullptr, 1.0,
                 false, nullptr, flags, false);
}

int grmhd_fixup(grmhd_ctx* ctx, double* P, const int8_t* flags, int32_t halo_sides) {
  if (!ctx) return GRMHD_EINVAL;
  if (!P || !flags) return fail(ctx, GRMHD_EINVAL, "fixup: NULL argument");
  if (halo_sides & ~63) return fail(ctx, GRMHD_EINVAL, "fixup: halo_sides has bits beyond the six sides");
  for (int d = 0; d < 3; ++d)
    if (ctx->up.periodic[d] && ((halo_sides >> (2 * d)) & 3))
      return fail(ctx, GRMHD_EINVAL, "fixup: a periodic direction cannot have halo sides");
  ProfScope ps(ctx->prof, ctx->stream, GRMHD_K_FIXUP);
  HIP_OR_FAIL(ctx, launch_fixup(ctx->d, ctx->t, ctx->up, P, flags, ctx->ctr, halo_sides, ctx->stream), "fixup");
  return GRMHD_OK;
}

int grmhd_speeds(grmhd_ctx* ctx, double ctop[3]) {
  if (!ctx || !ctop) return GRMHD_EINVAL;
  return read_speeds(ctx, ctop);
}

int grmhd_courant_dt(const grmhd_ctx* ctx, const double* ctop, int32_t nparts, double* dt) {
  if (!ctx || !ctop || !dt || nparts < 1) return GRMHD_EINVAL;
  double v[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < nparts; ++q)
    for (int d = 0; d < 3; ++d) {
      const double c = ctop[3 * q + d];
      if (!std::isfinite(c)) return GRMHD_ESTATE;
      if (c < 0.0) return GRMHD_EINVAL;
      v[d] = std::fmax(v[d], c);
    }
  *dt = courant_dt(ctx->p.cfl, v, ctx->dx);
  return GRMHD_OK;
}

int grmhd_divb_noalloc(grmhd_ctx* ctx, const double* P, double* max_divb) {
  if (!ctx) return GRMHD_EINVAL;
  if (!P || !max_divb) return fail(ctx, GRMHD_EINVAL, "divb_noalloc: NULL argument");
  const long long need = divb_blocks(ctx->d);
  if (need > DIVB_NOALLOC_PARTS)
    return fail(ctx, GRMHD_EINVAL,
                "divb_noalloc: the grid needs " + std::to_string(need) + " partial maxima, the static scratch holds " +
                    std::to_string(DIVB_NOALLOC_PARTS) + " (ceil(n1/64) ceil(n2/4) n3 must not exceed it)");
  if (!ctx->noalloc) return fail(ctx, GRMHD_EDEVICE, "divb_noalloc: no static scratch on this device");
  HIP_OR_FAIL(ctx, launch_divb_noalloc(ctx->p, ctx->d, ctx->t, P, ctx->noalloc, ctx->stream), "divb_noalloc");
  HIP_OR_FAIL(ctx, hipMemcpyAsync(max_divb, ctx->noalloc + DIVB_NOALLOC_PARTS, sizeof(double), hipMemcpyDeviceToHost,
                                  ctx->stream),
              "copy");
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
  return GRMHD_OK;
}

int grmhd_step_failures(grmhd_ctx* ctx, int64_t* n_fail) {
  if (!ctx || !n_fail) return GRMHD_EINVAL;
  unsigned int nf = 0;
  HIP_OR_FAIL(ctx, hipMemcpyAsync(&nf, &ctx->ctr->fail_total, sizeof(nf), hipMemcpyDeviceToHost, ctx->stream),
              "copy");
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
  *n_fail = nf;
  return GRMHD_OK;
}

int grmhd_divb(grmhd_ctx* ctx, const double* P, double* max_divb) {
  if (!ctx) return GRMHD_EINVAL;
  if (!P || !max_divb) return fail(ctx, GRMHD_EINVAL, "divb: NULL argument");
  HIP_OR_FAIL(ctx, launch_divb(ctx->p, ctx->d, ctx->t, P, ctx->ctr, ctx->stream), "divb");
  unsigned long long bits = 0;
  HIP_OR_FAIL(ctx, hipMemcpyAsync(&bits, &ctx->ctr->divb, sizeof(bits), hipMemcpyDeviceToHost, ctx->stream), "copy");
  HIP_OR_FAIL(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
  std::memcpy(max_divb, &bits, sizeof(double));
  return GRMHD_OK;
}

}  // extern "C"
