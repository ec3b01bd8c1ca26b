// Host-side launchers of the library's kernels (one translation unit each).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

struct Tables {
  double* cent;   // [N_CENT][p2][p1]
  double* f1;     // [N_FACE][p2][p1]
  double* f2;
  float* centf;   // float copies of the first N_FACE components (mixed precision)
  float* f1f;
  float* f2f;
};

// device counters kept by a context
struct Counters {
  unsigned long long ctop[3];  // max LLF speed per direction (double bits)
  unsigned long long divb;     // max |div B| (double bits)
  unsigned int fail;           // failed inversions of the current substep
  unsigned int fail_total;     // failed inversions since the last reset
};

// physical constants the update kernels need
struct UpdateParams {
  double gam;
  double sigma_max, beta_min, uorho_max, gamma_max;
  double dx1, dx2, dx3;
  int floors;
  int polar_lo, polar_hi;  // x2 boundaries are polar axes
};

hipError_t launch_geometry(const grmhd_problem& p, const Dims& d, const Tables& t, hipStream_t s);

hipError_t launch_fill_ghosts(const grmhd_problem& p, const Dims& d, const Tables& t, double* P,
                              const double* dirichlet_src, hipStream_t s);

// face fluxes in direction dir (1..3) of state P; F is double (fp64) or float
// (mixed). ctop may be null.
hipError_t launch_sweep(int dir, int recon, bool mixed, const Dims& d, const Tables& t, double gam,
                        const double* P, void* F, unsigned long long* ctop, hipStream_t s);

hipError_t launch_update(bool mixed, const Dims& d, const Tables& t, const UpdateParams& up,
                         const void* F1, const void* F2, const void* F3, const double* Pb,
                         const double* Ps, double* Pout, int8_t* flags, double dt,
                         Counters* ctr, hipStream_t s);

hipError_t launch_fixup(const Dims& d, const Tables& t, const UpdateParams& up, double* P,
                        const int8_t* flags, const Counters* ctr, hipStream_t s);

hipError_t launch_prim_to_cons(const Dims& d, const Tables& t, double gam, const double* P,
                               double* U, hipStream_t s);

hipError_t launch_cons_to_prim(const Dims& d, const Tables& t, const UpdateParams& up,
                               const double* U, double* P, int8_t* flags, Counters* ctr,
                               hipStream_t s);

hipError_t launch_divb(const grmhd_problem& p, const Dims& d, const Tables& t, const double* P,
                       Counters* ctr, hipStream_t s);

// zero the counters selected by mask (1: ctop, 2: divb, 4: fail, 8: fail_total)
hipError_t launch_reset(Counters* ctr, int mask, hipStream_t s);
