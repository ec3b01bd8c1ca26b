// Internal definition of a context (shared by the host-side translation units).
#pragma once

#include <string>
#include <vector>

#include "kernels.h"

struct ProfRecord {
  int kernel;
  hipEvent_t start, stop;
};

struct grmhd_ctx {
  bool profiling = false;
  std::vector<ProfRecord> prof;      // records since the last clear
  std::vector<hipEvent_t> event_pool;  // events of cleared records, for reuse
  grmhd_problem p;
  Dims d;
  hipStream_t stream;
  int device;
  bool mixed;
  Tables t;
  double* Ph;
  void* F[3];
  int8_t* flags;
  Counters* ctr;
  UpdateParams up;
  double dx[3];
  std::string err;
};

