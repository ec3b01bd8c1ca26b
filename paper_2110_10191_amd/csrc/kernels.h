// Host-side launchers of the library's kernels (one translation unit each).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

// Geometry tables over the padded (x1, x2) points (2D) or (x1, x2, x3) points
// (3D, Dims::tk != 0), ts points a component: the centre table one plane per
// component, [N_CENT][points]; the face tables two components interleaved
// per point, [N_FACE / 2][points][2] (pair_index), so the face-flux pass
// loads them two at a time. 2D tables hold the x3-face table too (the centre
// values, the metric not depending on x3).
struct Tables {
  double* cent;   // centre table, N_CENT components
  double* f1;     // x1-, x2-, x3-face tables, N_FACE components in pairs
  double* f2;
  double* f3;
  float* f1f;     // float copies of the face tables (mixed precision)
  float* f2f;
  float* f3f;
};

// device counters kept by a context
struct Counters {
  unsigned long long ctop[3];  // max LLF speed per direction (double bits)
  unsigned long long divb;     // max |div B| (double bits)
  unsigned int fail;           // failed inversions of the current substep
  unsigned int fail_total;     // failed inversions since the last reset
  unsigned int bad;            // non-finite values stored in the state since the last reset
  double dt;                   // step size kept on the device (grmhd_run)
  int status;                  // 1 once a non-finite speed met the device dt rule
};

// physical constants the update kernels need
struct UpdateParams {
  double gam;
  double sigma_max, beta_min, uorho_max, gamma_max;
  double dx1, dx2, dx3;
  double idx1, idx2, idx3;  // 1 / dx_d
  int floors;
  int polar_lo, polar_hi;  // x2 boundaries are polar axes
  int periodic[3];         // direction d (0 = x1) is periodic
};

// ---------------------------------------------------------------------------
// batched launches: one grid per phase spans every job of a batch

// one job of a batch (lives in device memory)
struct JobDesc {
  grmhd_problem p;
  Dims d;
  Tables t;
  UpdateParams up;
  double* P;        // the job's state (caller-owned)
  double* Ph;       // half-step state
  void* F[3];       // face fluxes (double or float)
  int8_t* flags;
  Counters* ctr;
  double* dt;       // device scalar: the job's step size for the next step
  int* status;      // device scalar: set to 1 when a non-finite speed appears
  // electron heating (E null: the job has none)
  double* E;        // the job's entropies (caller-owned)
  double* Eh;       // half-step entropies
  double* Uk;       // advected sqrt(-g) rho u^t K of the current substep
  int heat_model;
  double fel;
};

enum { PH_GHOST = 0, PH_SWEEP, PH_UPDATE, PH_COUNT };

// offs[ph * (njobs + 1) + j] = first block of job j in phase ph; entry njobs = total
struct BatchView {
  const JobDesc* jobs;
  const int* offs;
  int njobs;
  int stx, sty, utx, uty;  // block tiles shared by every job of the batch
};

// A pointer read from the device job table is a generic pointer to the
// compiler, which then emits flat loads (slower, and counted against both the
// vector and the scalar memory counters). Every array here is device global
// memory: say so, so the loads stay global loads.
// (Through an integer: a direct generic -> global -> generic cast pair is
// folded away and the information lost.)
template <typename T>
__device__ inline T* global_ptr(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

__device__ inline int batch_job(const int* offs, int njobs, int b) {
  int lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (offs[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// per-phase block counts of one job (stencil phases are multiples of 8)
void job_phase_blocks(const Dims& d, int counts[PH_COUNT]);

// corrector = false: predictor (ghosts of P, fluxes of P, P_base = P -> P_h, dt/2);
// corrector = true: ghosts of P_h, fluxes of P_h, (P, P_h) -> P with dt.
// totals[ph] = grid size of phase ph over the batch.
hipError_t launch_batch_ghosts(const BatchView& bv, const int* totals, bool corrector, hipStream_t s);
// the face fluxes of all three directions of every job
hipError_t launch_batch_sweeps(const BatchView& bv, const int* totals, int recon, bool mixed, bool corrector,
                               bool want_ctop, hipStream_t s);
// which: 1 the update, 2 the fixup, 3 both
hipError_t launch_batch_update(const BatchView& bv, const int* totals, bool mixed, bool corrector, int which,
                               hipStream_t s);
hipError_t launch_batch_reset(const BatchView& bv, int mask, hipStream_t s);
// electron passes of the jobs that have entropies (the others' blocks return
// at once): which 1 the scalar ghosts (ghost phase grids), 2 the advection, 3
// the heating (update phase grid)
hipError_t launch_batch_electrons(const BatchView& bv, const int* totals, bool mixed, int recon, bool corrector,
                                  int which, hipStream_t s);
hipError_t launch_batch_scalar_ghosts(const BatchView& bv, const int* totals, bool corrector, hipStream_t s);
// dt <- min(cfl / sum_d(ctop_d / dx_d), 1.3 dt) per job, on the device
hipError_t launch_batch_dt(const BatchView& bv, hipStream_t s);

hipError_t launch_geometry(const grmhd_problem& p, const Dims& d, const Tables& t, hipStream_t s);

// the step-size rule dt <- min(cfl / sum_d(ctop_d / dx_d), 1.3 dt) on the
// counters of the previous step (on = 0: not applied)
struct DtRule {
  int on;
  double cfl;
  double dx[3];
};

// with ctr: block 0 first applies dt_rule (when on) and then clears the
// counters of reset_mask, before any kernel after the fill counts into them
hipError_t launch_fill_ghosts(const grmhd_problem& p, const Dims& d, const Tables& t, double* P,
                              const double* dirichlet_src, hipStream_t s, Counters* ctr = nullptr,
                              int reset_mask = 0, DtRule dt_rule = DtRule{});

// face fluxes of all three directions of state P into F[0..2] (double for
// fp64, float for mixed) with the problem's reconstruction and gamma;
// Cartesian Kerr-Schild computes its face geometry instead of reading the
// face tables; ctop (may be null) receives the per-direction maximum signal
// speeds; sweep_blocks: the launch's grid size
unsigned sweep_blocks(const Dims& d);
hipError_t launch_sweeps(const grmhd_problem& p, bool mixed, const Dims& d, const Tables& t, const double* P,
                         void* const* F, unsigned long long* ctop, hipStream_t s);

// the step is dt, or dt_scale * *dt_dev when dt_dev is not null; cks (the
// problem, Cartesian Kerr-Schild only): the update computes the centre
// metric in closed form instead of reading it
hipError_t launch_update(bool mixed, const Dims& d, const Tables& t, const UpdateParams& up,
                         const void* F1, const void* F2, const void* F3, const double* Pb,
                         const double* Ps, double* Pout, int8_t* flags, double dt,
                         const double* dt_dev, double dt_scale, Counters* ctr, hipStream_t s,
                         const grmhd_problem* cks = nullptr);

// ctr->dt <- min(cfl / sum_d(ctop_d / dx_d), 1.3 ctr->dt) on the device
hipError_t launch_ctx_dt(Counters* ctr, double cfl, double dx1, double dx2, double dx3, hipStream_t s);

// halo: bit 2 d + side set where the ghost layer on that side of direction d
// holds a neighbouring part's zones (values and failure flags) for the fixup
hipError_t launch_fixup(const Dims& d, const Tables& t, const UpdateParams& up, double* P,
                        const int8_t* flags, Counters* ctr, int halo, hipStream_t s);

hipError_t launch_prim_to_cons(const Dims& d, const Tables& t, double gam, const double* P,
                               double* U, hipStream_t s);

hipError_t launch_cons_to_prim(const Dims& d, const Tables& t, const UpdateParams& up,
                               const double* U, double* P, int8_t* flags, Counters* ctr,
                               hipStream_t s);

hipError_t launch_divb(const grmhd_problem& p, const Dims& d, const Tables& t, const double* P,
                       Counters* ctr, hipStream_t s);

// div B without library-owned memory: per-block maxima in the device-resident
// static scratch (DIVB_NOALLOC_PARTS slots, then the result at slot
// DIVB_NOALLOC_PARTS). noalloc_scratch gives that array's address on the
// device (which must be current); divb_blocks the number of slots a grid needs.
constexpr int DIVB_NOALLOC_PARTS = 65536;
long long divb_blocks(const Dims& d);
hipError_t noalloc_scratch(int device, double** ptr);
hipError_t launch_divb_noalloc(const grmhd_problem& p, const Dims& d, const Tables& t, const double* P,
                               double* scr, hipStream_t s);

// electron heating: the ghost zones of the two entropies (the primitives'
// rules without the axis sign change and the inflow fix); the advection of
// U_K = sqrt(-g) rho u^t K from the face mass fluxes (F of double or float);
// the u ceiling and the heating of the new state. The advection's step is dt,
// or dt_scale * *dt_dev when dt_dev is not null.
hipError_t launch_fill_scalar_ghosts(const grmhd_problem& p, const Dims& d, double* E, const double* dirichlet_src,
                                     hipStream_t s);
hipError_t launch_scalar_advect(bool mixed, int recon, const Dims& d, const Tables& t, const UpdateParams& up,
                                const void* F1, const void* F2, const void* F3, const double* Pb, const double* Eb,
                                const double* Es, double* Uk, double dt, const double* dt_dev, double dt_scale,
                                hipStream_t s);
hipError_t launch_electron_heat(const Dims& d, const Tables& t, double gam, double* P, const double* Uk, double* E,
                                int model, double fel, Counters* ctr, hipStream_t s);

// zero the counters selected by mask (1: ctop, 2: divb, 4: fail, 8: fail_total and bad)
hipError_t launch_reset(Counters* ctr, int mask, hipStream_t s);
