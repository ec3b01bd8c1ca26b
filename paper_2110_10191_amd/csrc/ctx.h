// Internal definition of a context (shared by the host-side translation units).
#pragma once

#include <string>
#include <vector>

#include "kernels.h"

struct ProfRecord {
  int kernel;
  hipEvent_t start, stop;
};

// Event timing of kernel launches: records since the last clear, and the
// events of cleared records kept for reuse.
struct Profiler {
  bool on = false;
  unsigned mask = ~0u;  // kernel classes bracketed while on (bit GRMHD_K_*)
  std::vector<ProfRecord> rec;
  std::vector<hipEvent_t> pool;

  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void clear() {
    for (auto& r : rec) {
      pool.push_back(r.start);
      pool.push_back(r.stop);
    }
    rec.clear();
  }
  void destroy() {
    clear();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    pool.clear();
  }
  // summed ms and count of one kernel class; the stream must be synchronised
  hipError_t total(int kernel, double* ms, int64_t* n) const {
    double sum = 0.0;
    int64_t cnt = 0;
    for (const auto& r : rec) {
      if (r.kernel != kernel) continue;
      float t = 0.0f;
      const hipError_t e = hipEventElapsedTime(&t, r.start, r.stop);
      if (e != hipSuccess) return e;
      sum += t;
      ++cnt;
    }
    *ms = sum;
    *n = cnt;
    return hipSuccess;
  }
};

// brackets the launches made during its lifetime with events when profiling is on
struct ProfScope {
  Profiler& p;
  hipStream_t s;
  ProfRecord r{};
  bool on;
  ProfScope(Profiler& prof, hipStream_t stream, int kernel)
      : p(prof), s(stream), on(prof.on && ((prof.mask >> kernel) & 1u)) {
    if (!on) return;
    r.kernel = kernel;
    r.start = p.event();
    r.stop = p.event();
    if (!r.start || !r.stop) {
      on = false;
      return;
    }
    (void)hipEventRecord(r.start, s);
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(r.stop, s);
    p.rec.push_back(r);
  }
};

struct grmhd_ctx {
  Profiler prof;
  grmhd_problem p;
  Dims d;
  hipStream_t stream;
  int device;
  bool mixed;
  Tables t;
  double* Ph;
  double* Eh;  // electron heating scratch (allocated on first use): half-step entropies
  double* Uk;  // and the advected sqrt(-g) rho u^t K of the current substep
  void* F[3];
  int8_t* flags;
  Counters* ctr;
  double* noalloc;  // this device's static scratch (grmhd_divb_noalloc), not owned
  UpdateParams up;
  double dx[3];
  std::string err;
};

// electron heating helpers shared by the context and batch calls: the model /
// fel check, and the context's scratch (half-step entropies and U_K),
// allocated and its half-step array cleared on first use
bool heat_args_ok(int32_t model, double fel);
hipError_t ctx_electron_scratch(grmhd_ctx* c);

