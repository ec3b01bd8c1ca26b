// Host side of the batch calls: many independent jobs advanced by one grid per
// kernel phase, one step of all active jobs captured once in a HIP graph.
//
// Per step (all active jobs at once):
//   reset(fail_total)
//   predictor: ghosts(P); reset(fail); sweeps(P); update(P -> P_h, dt/2); fixup
//   corrector: ghosts(P_h); reset(ctop, fail); sweeps(P_h) + ctop; update((P, P_h) -> P, dt); fixup
//   dt_j <- min(cfl / sum_d (ctop_d / dx_d), 1.3 dt_j)
// With electron heating (jobs given entropies E), each substep also fills
// the scalar ghosts after the fluid ghosts, advects the entropies after the
// sweeps and heats after the fixup, as a context's electron step does.
// Every job reads only its own dt, counters and arrays, so its evolution is
// the same alone or in any mix.
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

struct grmhd_batch {
  std::vector<grmhd_ctx*> ctx;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int recon = 0;
  bool mixed = false;
  JobDesc* d_jobs = nullptr;
  int* d_offs = nullptr;
  double* d_dt = nullptr;
  int* d_status = nullptr;
  bool dt_set = false;
  // configuration the current graph was captured for
  std::vector<double*> cur_P;
  std::vector<int32_t> cur_active;
  std::vector<double*> cur_E;      // electron entropies per job (null: none)
  std::vector<int32_t> cur_model;
  std::vector<double> cur_fel;
  bool electrons = false;          // some active job has entropies
  int totals[PH_COUNT] = {0};
  int nactive = 0;
  int stx = TILE_X, sty = SWEEP_TILE_Y, utx = TILE_X, uty = TILE_Y;  // tiles of every job
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  Profiler prof;  // when on, steps run eagerly with each launch bracketed by events
  std::string err;
};

namespace {

thread_local std::string g_batch_error;

int bfail(grmhd_batch* b, int status, const std::string& msg) {
  if (b) b->err = msg;
  else g_batch_error = msg;
  return status;
}

#define BHIP(b, call, where)                                                                  \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) return bfail(b, GRMHD_EDEVICE, std::string(where) + ": " + hipGetErrorString(e_)); \
  } while (0)

void drop_graph(grmhd_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// enqueue one step of every job in the current job table (events around the
// launches only when profiling, which never happens under capture)
hipError_t enqueue_step(grmhd_batch* b) {
  const BatchView bv{b->d_jobs, b->d_offs, b->nactive, b->stx, b->sty, b->utx, b->uty};
  hipStream_t s = b->stream;
  hipError_t e;
  if ((e = launch_batch_reset(bv, 8, s)) != hipSuccess) return e;
  for (int corr = 0; corr < 2; ++corr) {
    {
      ProfScope ps(b->prof, s, GRMHD_K_GHOSTS);
      if ((e = launch_batch_ghosts(bv, b->totals, corr == 1, s)) != hipSuccess) return e;
    }
    if (b->electrons) {
      ProfScope ps(b->prof, s, GRMHD_K_ELECTRONS);
      if ((e = launch_batch_electrons(bv, b->totals, b->mixed, b->recon, corr == 1, 1, s)) != hipSuccess) return e;
    }
    if ((e = launch_batch_reset(bv, corr ? (1 | 4) : 4, s)) != hipSuccess) return e;
    {
      ProfScope ps(b->prof, s, GRMHD_K_SWEEPS);
      if ((e = launch_batch_sweeps(bv, b->totals, b->recon, b->mixed, corr == 1, corr == 1, s)) != hipSuccess)
        return e;
    }
    if (b->electrons) {
      // before the update: in the corrector it overwrites the base state
      ProfScope ps(b->prof, s, GRMHD_K_ELECTRONS);
      if ((e = launch_batch_electrons(bv, b->totals, b->mixed, b->recon, corr == 1, 2, s)) != hipSuccess) return e;
    }
    {
      ProfScope ps(b->prof, s, GRMHD_K_UPDATE);
      if ((e = launch_batch_update(bv, b->totals, b->mixed, corr == 1, 1, s)) != hipSuccess) return e;
    }
    {
      ProfScope ps(b->prof, s, GRMHD_K_FIXUP);
      if ((e = launch_batch_update(bv, b->totals, b->mixed, corr == 1, 2, s)) != hipSuccess) return e;
    }
    if (b->electrons) {
      ProfScope ps(b->prof, s, GRMHD_K_ELECTRONS);
      if ((e = launch_batch_electrons(bv, b->totals, b->mixed, b->recon, corr == 1, 3, s)) != hipSuccess) return e;
    }
  }
  return launch_batch_dt(bv, s);
}

// E, model, fel: electron heating per job (E null, or E[j] null: none)
int configure(grmhd_batch* b, double* const* P, double* const* E, const int32_t* model, const double* fel,
              const int32_t* active) {
  const int n = (int)b->ctx.size();
  std::vector<JobDesc> jobs;
  std::vector<int> counts;  // [job][phase]
  bool electrons = false;
  for (int j = 0; j < n; ++j) {
    if (active && !active[j]) continue;
    if (!P[j]) return bfail(b, GRMHD_EINVAL, "batch_step: NULL state for an active job");
    grmhd_ctx* c = b->ctx[j];
    const bool ej = E && E[j];
    if (ej) {
      if (!heat_args_ok(model[j], fel[j]))
        return bfail(b, GRMHD_EINVAL, "batch_step_electrons: unknown heating model or fel outside [0, 1]");
      const hipError_t e = ctx_electron_scratch(c);
      if (e != hipSuccess)
        return bfail(b, e == hipErrorOutOfMemory ? GRMHD_ENOMEM : GRMHD_EDEVICE,
                     std::string("electron scratch: ") + hipGetErrorString(e));
      // the scratch is cleared on the context's stream
      BHIP(b, hipStreamSynchronize(c->stream), "synchronize");
      electrons = true;
    }
    JobDesc jd;
    std::memset(&jd, 0, sizeof(jd));
    jd.p = c->p;
    jd.d = c->d;
    jd.d.stx = b->stx;
    jd.d.sty = b->sty;
    jd.d.utx = b->utx;
    jd.d.uty = b->uty;
    jd.t = c->t;
    jd.up = c->up;
    jd.P = P[j];
    jd.Ph = c->Ph;
    jd.F[0] = c->F[0];
    jd.F[1] = c->F[1];
    jd.F[2] = c->F[2];
    jd.flags = c->flags;
    jd.ctr = c->ctr;
    jd.dt = b->d_dt + j;
    jd.status = b->d_status + j;
    if (ej) {
      jd.E = E[j];
      jd.Eh = c->Eh;
      jd.Uk = c->Uk;
      jd.heat_model = model[j];
      jd.fel = fel[j];
    }
    jobs.push_back(jd);
    int cnt[PH_COUNT];
    job_phase_blocks(jd.d, cnt);
    counts.insert(counts.end(), cnt, cnt + PH_COUNT);
  }
  const int na = (int)jobs.size();
  std::vector<int> offs((size_t)PH_COUNT * (na + 1), 0);
  for (int ph = 0; ph < PH_COUNT; ++ph) {
    long long acc = 0;
    for (int j = 0; j < na; ++j) {
      offs[(size_t)ph * (na + 1) + j] = (int)acc;
      acc += counts[(size_t)j * PH_COUNT + ph];
    }
    if (acc >= (1ll << 31)) return bfail(b, GRMHD_EINVAL, "batch too large for one grid");
    offs[(size_t)ph * (na + 1) + na] = (int)acc;
    b->totals[ph] = (int)acc;
  }
  BHIP(b, hipStreamSynchronize(b->stream), "synchronize");
  drop_graph(b);
  b->nactive = na;
  b->cur_P.assign(P, P + n);
  b->cur_active.assign(n, 1);
  if (active) b->cur_active.assign(active, active + n);
  b->cur_E.assign(n, nullptr);
  b->cur_model.assign(n, 0);
  b->cur_fel.assign(n, 0.0);
  if (E)
    for (int j = 0; j < n; ++j)
      if (E[j]) {
        b->cur_E[j] = E[j];
        b->cur_model[j] = model[j];
        b->cur_fel[j] = fel[j];
      }
  b->electrons = electrons;
  if (na == 0) return GRMHD_OK;
  // on the batch's stream, which may be a non-blocking one: a copy on the
  // null stream is not ordered before the graph launched on it, and a copy
  // from pageable memory may return before its data has landed
  BHIP(b, hipMemcpyAsync(b->d_jobs, jobs.data(), sizeof(JobDesc) * na, hipMemcpyHostToDevice, b->stream),
       "upload jobs");
  BHIP(b, hipMemcpyAsync(b->d_offs, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice, b->stream),
       "upload offsets");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronize");
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "begin capture");
  const bool prof_on = b->prof.on;
  b->prof.on = false;
  hipError_t e = enqueue_step(b);
  b->prof.on = prof_on;
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bfail(b, GRMHD_EDEVICE, std::string("capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  }
  b->graph = g;
  BHIP(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "instantiate");
  return GRMHD_OK;
}

bool same_config(const grmhd_batch* b, double* const* P, double* const* E, const int32_t* model, const double* fel,
                 const int32_t* active) {
  const size_t n = b->ctx.size();
  if (b->cur_P.size() != n) return false;
  for (size_t j = 0; j < n; ++j) {
    const int32_t a = active ? (active[j] != 0) : 1;
    if (a != (b->cur_active[j] != 0)) return false;
    if (!a) continue;
    if (b->cur_P[j] != P[j]) return false;
    double* ej = E ? E[j] : nullptr;
    if (b->cur_E[j] != ej) return false;
    if (ej && (b->cur_model[j] != model[j] || b->cur_fel[j] != fel[j])) return false;
  }
  return true;
}

int batch_step(grmhd_batch* b, double* const* P, double* const* E, const int32_t* model, const double* fel,
               const int32_t* active, int32_t nsteps) {
  if (!P) return bfail(b, GRMHD_EINVAL, "batch_step: NULL state list");
  if (nsteps < 0) return bfail(b, GRMHD_EINVAL, "batch_step: nsteps < 0");
  if (!b->dt_set) return bfail(b, GRMHD_EINVAL, "batch_step: call grmhd_batch_set_dt first");
  if (!b->exec || !same_config(b, P, E, model, fel, active)) {
    const int st = configure(b, P, E, model, fel, active);
    if (st != GRMHD_OK) return st;
  }
  if (b->nactive == 0) return GRMHD_OK;
  if (b->prof.on) {
    for (int s = 0; s < nsteps; ++s) BHIP(b, enqueue_step(b), "step");
    return GRMHD_OK;
  }
  for (int s = 0; s < nsteps; ++s) BHIP(b, hipGraphLaunch(b->exec, b->stream), "graph launch");
  return GRMHD_OK;
}

}  // namespace

extern "C" {

int grmhd_batch_create(grmhd_ctx* const* jobs, int32_t n, void* hip_stream, grmhd_batch** out) {
  if (!out) return bfail(nullptr, GRMHD_EINVAL, "out is NULL");
  *out = nullptr;
  if (!jobs || n < 1) return bfail(nullptr, GRMHD_EINVAL, "need at least one job");
  for (int j = 0; j < n; ++j)
    if (!jobs[j]) return bfail(nullptr, GRMHD_EINVAL, "NULL context in the job list");
  for (int j = 1; j < n; ++j) {
    if (jobs[j]->device != jobs[0]->device) return bfail(nullptr, GRMHD_EINVAL, "jobs on different devices");
    if (jobs[j]->p.recon != jobs[0]->p.recon || jobs[j]->p.precision != jobs[0]->p.precision)
      return bfail(nullptr, GRMHD_EUNSUPPORTED, "jobs of one batch need the same recon and precision");
  }
  grmhd_batch* b = new grmhd_batch();
  b->ctx.assign(jobs, jobs + n);
  b->recon = jobs[0]->p.recon;
  b->mixed = jobs[0]->mixed;
  b->stx = jobs[0]->d.stx;
  b->sty = jobs[0]->d.sty;
  b->utx = jobs[0]->d.utx;
  b->uty = jobs[0]->d.uty;
  b->stream = (hipStream_t)hip_stream;
  hipError_t e = hipSuccess;
  if (!b->stream) {
    e = hipStreamCreate(&b->stream);
    b->own_stream = e == hipSuccess;
  }
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_jobs, sizeof(JobDesc) * n);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_offs, sizeof(int) * PH_COUNT * (n + 1));
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_dt, sizeof(double) * n);
  if (e == hipSuccess) e = hipMalloc((void**)&b->d_status, sizeof(int) * n);
  // cleared on the batch's stream, so that the clear is ordered before the
  // step sizes grmhd_batch_set_dt copies in on the same stream (a null-stream
  // memset is not ordered with a non-blocking stream and could land after
  // them, leaving a job a zero step)
  if (e == hipSuccess) e = hipMemsetAsync(b->d_status, 0, sizeof(int) * n, b->stream);
  if (e == hipSuccess) e = hipMemsetAsync(b->d_dt, 0, sizeof(double) * n, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    std::string m = std::string("batch set-up: ") + hipGetErrorString(e);
    grmhd_batch_free(b);
    return bfail(nullptr, e == hipErrorOutOfMemory ? GRMHD_ENOMEM : GRMHD_EDEVICE, m);
  }
  *out = b;
  return GRMHD_OK;
}

int grmhd_batch_set_dt(grmhd_batch* b, const double* dt) {
  if (!b || !dt) return GRMHD_EINVAL;
  for (size_t j = 0; j < b->ctx.size(); ++j)
    if (!(dt[j] > 0.0)) return bfail(b, GRMHD_EINVAL, "batch_set_dt: every dt must be > 0");
  BHIP(b, hipMemcpyAsync(b->d_dt, dt, sizeof(double) * b->ctx.size(), hipMemcpyHostToDevice, b->stream), "set dt");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronize");
  b->dt_set = true;
  return GRMHD_OK;
}

int grmhd_batch_get(grmhd_batch* b, double* dt, int32_t* status) {
  if (!b) return GRMHD_EINVAL;
  const size_t n = b->ctx.size();
  if (dt) BHIP(b, hipMemcpyAsync(dt, b->d_dt, sizeof(double) * n, hipMemcpyDeviceToHost, b->stream), "read dt");
  std::vector<int> st(n);
  if (status)
    BHIP(b, hipMemcpyAsync(st.data(), b->d_status, sizeof(int) * n, hipMemcpyDeviceToHost, b->stream), "read status");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronize");
  if (status)
    for (size_t j = 0; j < n; ++j) status[j] = st[j];
  return GRMHD_OK;
}

int grmhd_batch_step(grmhd_batch* b, double* const* P, const int32_t* active, int32_t nsteps) {
  if (!b) return GRMHD_EINVAL;
  return batch_step(b, P, nullptr, nullptr, nullptr, active, nsteps);
}

int grmhd_batch_step_electrons(grmhd_batch* b, double* const* P, double* const* E, const int32_t* model,
                               const double* fel, const int32_t* active, int32_t nsteps) {
  if (!b) return GRMHD_EINVAL;
  if (!E || !model || !fel) return bfail(b, GRMHD_EINVAL, "batch_step_electrons: NULL list");
  return batch_step(b, P, E, model, fel, active, nsteps);
}

int grmhd_batch_profile(grmhd_batch* b, int32_t enable) {
  if (!b) return GRMHD_EINVAL;
  if (enable) {
    BHIP(b, hipStreamSynchronize(b->stream), "synchronize");
    b->prof.clear();
  }
  b->prof.on = enable != 0;
  return GRMHD_OK;
}

int grmhd_batch_profile_read(grmhd_batch* b, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!b || !total_ms || !launches) return GRMHD_EINVAL;
  if (kernel < 0 || kernel >= GRMHD_K_COUNT) return bfail(b, GRMHD_EINVAL, "profile_read: unknown kernel");
  BHIP(b, hipStreamSynchronize(b->stream), "synchronize");
  BHIP(b, b->prof.total(kernel, total_ms, launches), "event time");
  return GRMHD_OK;
}

int grmhd_batch_free(grmhd_batch* b) {
  if (!b) return GRMHD_OK;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graph(b);
  b->prof.destroy();
  void* ptrs[] = {b->d_jobs, b->d_offs, b->d_dt, b->d_status};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return GRMHD_OK;
}

const char* grmhd_batch_last_error(const grmhd_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

}  // extern "C"
