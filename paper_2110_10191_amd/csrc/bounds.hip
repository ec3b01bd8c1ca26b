// Ghost zones, the div B monitor, counter resets and the per-job time step.
//
// Ghost fill (three ghost layers): the result of filling in the order x1
// (interior j, k), x2 (all i, interior k), x3 (all i, j), so corners are
// consistent, computed in one launch with each ghost taken straight from the
// interior zone it comes from (the electron-heating scalars follow the same
// rules without the inflow fix and the axis sign change):
//   periodic  - wrap;
//   outflow   - copy the nearest interior zone; where the copied radial
//               four-velocity points into the domain, u~1 is reset so u^1 = 0;
//   polar     - ghost row -1-m mirrors row m with u~2 and B2 negated;
//   dirichlet - the ghosts keep the caller's values (copied from the base state
//               into the half-step state).
#include <mutex>

#include "kernels.h"

namespace {

__device__ void reset_counters(Counters* c, int mask);
__device__ void device_dt(const unsigned long long* ctop, unsigned bad, const double* dx, double cfl, double* dt,
                          int* status);

constexpr int MAX_DEVICES = 64;  // devices the no-allocation scratch lookup keeps

__device__ inline int wrap(int x, int n) {
  int r = x % n;
  return r < 0 ? r + n : r;
}

// where an outflow ghost's u^1 points into the domain, set u~1 = c Gamma with
// c = alpha g^{t1}, Gamma the positive root of
// (1 - g11 c^2) G^2 - 2 c (g12 v2 + g13 v3) G - (1 + g_jk v^j v^k) = 0
// (q: the ghost's primitives)
__device__ void inflow_fix(double* q, const double* cent, int ts, int toff, int side) {
  Geo<double> g;
  load_geo(g, cent, ts, toff);
  const double v1 = q[2], v2 = q[3], v3 = q[4];
  const double lor = sqrt(lorentz_sq(g.gcov, v1, v2, v3));
  const double u1 = v1 - lor * g.alpha * g.gcon[1];
  const bool bad = side == 0 ? (u1 > 0.0) : (u1 < 0.0);
  if (!bad) return;
  const double c = g.alpha * g.gcon[1];
  const double qa = 1.0 - g.gcov[4] * c * c;
  if (!(qa > 0.0)) return;
  const double G = g.gcov[5] * v2 + g.gcov[6] * v3;
  const double H = g.gcov[7] * v2 * v2 + 2.0 * g.gcov[8] * v2 * v3 + g.gcov[9] * v3 * v3;
  const double root = (c * G + sqrt(c * c * G * G + qa * (1.0 + H))) / qa;
  q[2] = c * root;
}

// ---- bodies: idx is the thread index within one job's grid. NVAR variables of
// stride d.sv; SCALAR: advected scalars (no inflow fix, no sign change on the
// axis), otherwise the primitives.

// The value the fill in the order x1 (interior j, k), x2 (all i, interior k),
// x3 (all i, j) leaves in ghost cell (i, j, k), taken straight from the
// interior cell (or the Dirichlet source) it comes from: the x3 rule maps k to
// an interior plane, the x2 rule j to an interior row, the x1 rule i to an
// interior column, and the value changes on the way back in the fill's order
// (inflow fix at the x1 ghost, sign change across the axis). No cell is read
// that the same launch writes, so one launch does all three directions.
template <int NVAR, bool SCALAR>
__device__ void ghost_cell(const grmhd_problem& p, const Dims& d, const double* cent, double* P,
                           const double* dsrc, int i, int j, int k) {
  const int cg = cell_of(d, k, j, i);
  int sk = k, sj = j, si = i;
  if (k < 0 || k >= d.n3) {
    const int side = k < 0 ? 0 : 1, type = p.bc[2][side];
    if (type == GRMHD_BC_DIRICHLET) {
      if (dsrc != P)
        for (int v = 0; v < NVAR; ++v) P[v * d.sv + cg] = dsrc[v * d.sv + cg];
      return;
    }
    sk = type == GRMHD_BC_PERIODIC ? wrap(k, d.n3) : (side == 0 ? 0 : d.n3 - 1);
  }
  bool flip = false;
  if (j < 0 || j >= d.n2) {
    const int side = j < 0 ? 0 : 1, type = p.bc[1][side];
    if (type == GRMHD_BC_DIRICHLET) {
      // the x2 fill leaves the source's value at (i, j, sk)
      const int cs = cell_of(d, sk, j, i);
      if (dsrc != P || cs != cg)
        for (int v = 0; v < NVAR; ++v) P[v * d.sv + cg] = dsrc[v * d.sv + cs];
      return;
    }
    const int m = side == 0 ? -1 - j : j - d.n2;
    if (type == GRMHD_BC_PERIODIC) sj = wrap(j, d.n2);
    else if (type == GRMHD_BC_POLAR) sj = side == 0 ? m : d.n2 - 1 - m;
    else sj = side == 0 ? 0 : d.n2 - 1;
    flip = !SCALAR && type == GRMHD_BC_POLAR;
  }
  const double* from = P;
  int fix_side = -1;
  if (i < 0 || i >= d.n1) {
    const int side = i < 0 ? 0 : 1, type = p.bc[0][side];
    if (type == GRMHD_BC_DIRICHLET) {
      from = dsrc;  // the x1 fill leaves the source's value at (i, sj, sk)
    } else {
      si = type == GRMHD_BC_PERIODIC ? wrap(i, d.n1) : (side == 0 ? 0 : d.n1 - 1);
      if (!SCALAR && type == GRMHD_BC_OUTFLOW) fix_side = side;
    }
  }
  const int cs = cell_of(d, sk, sj, si);
  if (from == P && cs == cg) return;  // a Dirichlet ghost that keeps its value
  double q[NVAR];
  for (int v = 0; v < NVAR; ++v) q[v] = from[v * d.sv + cs];
  if constexpr (!SCALAR) {
    if (fix_side >= 0) inflow_fix(q, tab_plane(cent, d, sk), d.ts, tab_of(d, sj, i), fix_side);
    if (flip) {
      q[3] = -q[3];
      q[6] = -q[6];
    }
  }
  for (int v = 0; v < NVAR; ++v) P[v * d.sv + cg] = q[v];
}

// thread idx of the fused fill: the x1 ghosts at interior (j, k) (the six of a
// row side by side), then the x2 ghosts at every i and interior k, then the x3
// ghosts at every (i, j), i fastest
__host__ __device__ inline int ghost_threads(const Dims& d) {
  const int w = d.n1 + 2 * NG, h = d.n2 + 2 * NG;
  return 2 * NG * (d.n2 * d.n3 + w * d.n3 + w * h);
}

template <int NVAR = NV, bool SCALAR = false>
__device__ void ghost_fill_body(const grmhd_problem& p, const Dims& d, const double* cent, double* P,
                                const double* dsrc, int idx) {
  const int w = d.n1 + 2 * NG, h = d.n2 + 2 * NG;
  const int t1 = 2 * NG * d.n2 * d.n3, t2 = 2 * NG * w * d.n3, t3 = 2 * NG * w * h;
  int i, j, k;
  if (idx < t1) {
    const int t = idx % (2 * NG), rest = idx / (2 * NG);
    j = rest % d.n2;
    k = rest / d.n2;
    i = t < NG ? -1 - t : d.n1 + (t - NG);
  } else if ((idx -= t1) < t2) {
    i = idx % w - NG;
    const int rest = idx / w, t = rest % (2 * NG);
    k = rest / (2 * NG);
    j = t < NG ? -1 - t : d.n2 + (t - NG);
  } else if ((idx -= t2) < t3) {
    i = idx % w - NG;
    const int rest = idx / w, t = rest / h;
    j = rest % h - NG;
    k = t < NG ? -1 - t : d.n3 + (t - NG);
  } else {
    return;
  }
  ghost_cell<NVAR, SCALAR>(p, d, cent, P, dsrc, i, j, k);
}

// ---- single-job kernels

// all ghosts of a state in one launch; block 0 also takes the step size from
// the previous step's counters (dr.on) and then clears the counters of
// reset_mask (the step's ghost fill comes before the kernels that count)
__global__ __launch_bounds__(256) void ghost_fill_kernel(grmhd_problem p, Dims d, const double* __restrict__ cent,
                                                         double* P, const double* dsrc, Counters* ctr,
                                                         int reset_mask, DtRule dr) {
  if (ctr && blockIdx.x == 0 && threadIdx.x == 0) {
    if (dr.on) device_dt(ctr->ctop, ctr->bad, dr.dx, dr.cfl, &ctr->dt, &ctr->status);
    reset_counters(ctr, reset_mask);
  }
  ghost_fill_body(p, d, cent, P, dsrc, (int)(blockIdx.x * blockDim.x + threadIdx.x));
}

// the two advected entropies of the electron-heating step
__global__ __launch_bounds__(256) void scalar_ghost_fill_kernel(grmhd_problem p, Dims d, double* E, const double* dsrc) {
  ghost_fill_body<GRMHD_NSCALAR, true>(p, d, nullptr, E, dsrc, (int)(blockIdx.x * blockDim.x + threadIdx.x));
}

// ---- batched kernels: the block finds its job, then runs the same body

__global__ __launch_bounds__(256) void ghost_batch_kernel(BatchView bv, int corrector) {
  const int* offs = bv.offs + PH_GHOST * (bv.njobs + 1);
  const int jb = batch_job(offs, bv.njobs, (int)blockIdx.x);
  const JobDesc& J = bv.jobs[jb];
  const int b = (int)blockIdx.x - offs[jb];
  double* tgt = global_ptr(corrector ? J.Ph : J.P);
  const double* src = global_ptr(J.P);
  ghost_fill_body(J.p, J.d, global_ptr(J.t.cent), tgt, src, b * (int)blockDim.x + (int)threadIdx.x);
}

// the electron entropies of the jobs that have them: predictor fills E,
// corrector E_h (Dirichlet ghosts from E)
__global__ __launch_bounds__(256) void scalar_ghost_batch_kernel(BatchView bv, int corrector) {
  const int* offs = bv.offs + PH_GHOST * (bv.njobs + 1);
  const int jb = batch_job(offs, bv.njobs, (int)blockIdx.x);
  const JobDesc& J = bv.jobs[jb];
  if (!J.E) return;
  const int b = (int)blockIdx.x - offs[jb];
  double* tgt = global_ptr(corrector ? J.Eh : J.E);
  const double* src = global_ptr(J.E);
  ghost_fill_body<GRMHD_NSCALAR, true>(J.p, J.d, nullptr, tgt, src, b * (int)blockDim.x + (int)threadIdx.x);
}

// |corner-centred divergence of sqrt(-g) B| at corner (i, j, k), which sits at
// (i-1/2, j-1/2, k-1/2); 0 for corners outside the grid or on a non-periodic
// edge, +inf for a NaN
__device__ double divb_at(const grmhd_problem& p, const Dims& d, const double* __restrict__ cent,
                          const double* __restrict__ P, int i, int j, int k) {
  const bool p1 = p.bc[0][0] == GRMHD_BC_PERIODIC, p2 = p.bc[1][0] == GRMHD_BC_PERIODIC,
             p3 = p.bc[2][0] == GRMHD_BC_PERIODIC;
  const bool ok = i < d.n1 && j < d.n2 && k < d.n3 && (p1 || i > 0) && (p2 || j > 0) && (p3 || k > 0);
  if (!ok) return 0.0;
  const int im = wrap(i - 1, d.n1), jm = wrap(j - 1, d.n2), km = wrap(k - 1, d.n3);
  // G_d(kk, jj, ii) = sqrt(-g) B^d
  auto G = [&](int v, int kk, int jj, int ii) {
    return tab_plane(cent, d, kk)[T_GDET * d.ts + tab_of(d, jj, ii)] * P[(5 + v) * d.sv + cell_of(d, kk, jj, ii)];
  };
  // sum over the two transverse offsets, differencing along the direction
  const double s1 = (G(0, k, j, i) - G(0, k, j, im)) + (G(0, k, jm, i) - G(0, k, jm, im)) +
                    (G(0, km, j, i) - G(0, km, j, im)) + (G(0, km, jm, i) - G(0, km, jm, im));
  const double s2 = (G(1, k, j, i) - G(1, k, jm, i)) + (G(1, k, j, im) - G(1, k, jm, im)) +
                    (G(1, km, j, i) - G(1, km, jm, i)) + (G(1, km, j, im) - G(1, km, jm, im));
  const double s3 = (G(2, k, j, i) - G(2, km, j, i)) + (G(2, k, j, im) - G(2, km, j, im)) +
                    (G(2, k, jm, i) - G(2, km, jm, i)) + (G(2, k, jm, im) - G(2, km, jm, im));
  const double dx1 = (p.x1max - p.x1min) / p.n1, dx2 = (p.x2max - p.x2min) / p.n2,
               dx3 = (p.x3max - p.x3min) / p.n3;
  const double val = fabs(s1 / (4.0 * dx1) + s2 / (4.0 * dx2) + s3 / (4.0 * dx3));
  return val != val ? __builtin_inf() : val;
}

// one 64 x 4 block per (x1, x2) tile and x3 plane; the maximum over the block
// goes into *out by one atomic max
__global__ void divb_kernel(grmhd_problem p, Dims d, const double* __restrict__ cent,
                            const double* __restrict__ P, unsigned long long* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  block_max_to(divb_at(p, d, cent, P, i, j, (int)blockIdx.z), out);
}

// The same blocks, each writing its maximum to its own slot of part[] (no
// atomics, nothing to clear beforehand); then one block reduces the slots.
__global__ __launch_bounds__(256) void divb_part_kernel(grmhd_problem p, Dims d, const double* __restrict__ cent,
                                                        const double* __restrict__ P, double* __restrict__ part) {
  __shared__ double wmax[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y * blockDim.y + threadIdx.y;
  const int tid = threadIdx.x + blockDim.x * threadIdx.y;
  const double v = wave_max(divb_at(p, d, cent, P, i, j, (int)blockIdx.z));
  if ((tid & 63) == 0) wmax[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    const int b = (int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z));
    part[b] = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
  }
}

__global__ __launch_bounds__(256) void max_reduce_kernel(const double* __restrict__ part, int n,
                                                         double* __restrict__ out) {
  __shared__ double wmax[4];
  double m = 0.0;
  for (int q = (int)threadIdx.x; q < n; q += 256) m = fmax(m, part[q]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
}

// Scratch of the no-allocation div B call: one double per block of
// divb_part_kernel, and the result after them. One copy per device, held
// until the process ends; the host reaches it only through the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[DIVB_NOALLOC_PARTS + 32];

__device__ void reset_counters(Counters* c, int mask) {
  if (mask & 1) c->ctop[0] = c->ctop[1] = c->ctop[2] = 0ull;
  if (mask & 2) c->divb = 0ull;
  if (mask & 4) c->fail = 0u;
  if (mask & 8) {
    c->fail_total = 0u;
    c->bad = 0u;
  }
}

__global__ void reset_kernel(Counters* c, int mask) {
  if (threadIdx.x != 0) return;
  reset_counters(c, mask);
}

__global__ void reset_batch_kernel(BatchView bv, int mask) {
  const int jb = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (jb >= bv.njobs) return;
  reset_counters(bv.jobs[jb].ctr, mask);
}

// dt <- min(cfl / sum_d (ctop_d / dx_d), 1.3 dt) (1.3 dt when every speed is
// 0); a non-finite speed, or a non-finite value stored in the state during the
// step (bad != 0), keeps dt and raises the status flag. The same operations, in
// the same order, as the host rule after grmhd_step.
__device__ void device_dt(const unsigned long long* ctop, unsigned bad, const double* dx, double cfl, double* dt,
                          int* status) {
  double sum = 0.0;
  bool finite = bad == 0u;
  for (int d = 0; d < 3; ++d) {
    const double c = __longlong_as_double((long long)ctop[d]);
    finite = finite && isfinite(c);
    sum += c / dx[d];
  }
  if (!finite) {
    *status = 1;
    return;
  }
  const double dn = sum > 0.0 ? cfl / sum : __builtin_inf();
  *dt = fmin(dn, 1.3 * *dt);
}

__global__ void dt_ctx_kernel(Counters* ctr, double cfl, double dx1, double dx2, double dx3) {
  if (threadIdx.x != 0) return;
  const double dx[3] = {dx1, dx2, dx3};
  device_dt(ctr->ctop, ctr->bad, dx, cfl, &ctr->dt, &ctr->status);
}

__global__ void dt_batch_kernel(BatchView bv) {
  const int jb = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (jb >= bv.njobs) return;
  const JobDesc& J = bv.jobs[jb];
  const double dx[3] = {J.up.dx1, J.up.dx2, J.up.dx3};
  device_dt(J.ctr->ctop, J.ctr->bad, dx, J.p.cfl, J.dt, J.status);
}

dim3 divb_grid(const Dims& d) { return dim3((d.n1 + 63) / 64, (d.n2 + 3) / 4, d.n3); }

}  // namespace

hipError_t launch_fill_ghosts(const grmhd_problem& p, const Dims& d, const Tables& t, double* P,
                              const double* dsrc, hipStream_t s, Counters* ctr, int reset_mask, DtRule dt_rule) {
  const int n = ghost_threads(d);
  hipLaunchKernelGGL(ghost_fill_kernel, dim3((n + 255) / 256), dim3(256, 1, 1), 0, s, p, d, t.cent, P, dsrc, ctr,
                     reset_mask, dt_rule);
  return hipGetLastError();
}

hipError_t launch_fill_scalar_ghosts(const grmhd_problem& p, const Dims& d, double* E, const double* dsrc,
                                     hipStream_t s) {
  const int n = ghost_threads(d);
  hipLaunchKernelGGL(scalar_ghost_fill_kernel, dim3((n + 255) / 256), dim3(256, 1, 1), 0, s, p, d, E, dsrc);
  return hipGetLastError();
}

hipError_t launch_divb(const grmhd_problem& p, const Dims& d, const Tables& t, const double* P,
                       Counters* ctr, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, ctr, 2);
  hipLaunchKernelGGL(divb_kernel, divb_grid(d), dim3(64, 4, 1), 0, s, p, d, t.cent, P, &ctr->divb);
  return hipGetLastError();
}

long long divb_blocks(const Dims& d) {
  const dim3 g = divb_grid(d);
  return (long long)g.x * g.y * g.z;
}

// the address of scratch on each device, looked up once per device (with that
// device current) and kept for the life of the process
hipError_t noalloc_scratch(int device, double** ptr) {
  static std::mutex mu;
  static double* addr[MAX_DEVICES] = {};
  *ptr = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = (double*)q;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_divb_noalloc(const grmhd_problem& p, const Dims& d, const Tables& t, const double* P,
                               double* scr, hipStream_t s) {
  const int n = (int)divb_blocks(d);
  hipLaunchKernelGGL(divb_part_kernel, divb_grid(d), dim3(64, 4, 1), 0, s, p, d, t.cent, P, scr);
  hipLaunchKernelGGL(max_reduce_kernel, dim3(1), dim3(256), 0, s, scr, n, scr + DIVB_NOALLOC_PARTS);
  return hipGetLastError();
}

hipError_t launch_ctx_dt(Counters* ctr, double cfl, double dx1, double dx2, double dx3, hipStream_t s) {
  hipLaunchKernelGGL(dt_ctx_kernel, dim3(1), dim3(64), 0, s, ctr, cfl, dx1, dx2, dx3);
  return hipGetLastError();
}

hipError_t launch_reset(Counters* ctr, int mask, hipStream_t s) {
  hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, s, ctr, mask);
  return hipGetLastError();
}

hipError_t launch_batch_ghosts(const BatchView& bv, const int* totals, bool corrector, hipStream_t s) {
  hipLaunchKernelGGL(ghost_batch_kernel, dim3(totals[PH_GHOST]), dim3(256), 0, s, bv, corrector ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_batch_scalar_ghosts(const BatchView& bv, const int* totals, bool corrector, hipStream_t s) {
  hipLaunchKernelGGL(scalar_ghost_batch_kernel, dim3(totals[PH_GHOST]), dim3(256), 0, s, bv, corrector ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_batch_reset(const BatchView& bv, int mask, hipStream_t s) {
  hipLaunchKernelGGL(reset_batch_kernel, dim3((bv.njobs + 63) / 64), dim3(64), 0, s, bv, mask);
  return hipGetLastError();
}

hipError_t launch_batch_dt(const BatchView& bv, hipStream_t s) {
  hipLaunchKernelGGL(dt_batch_kernel, dim3((bv.njobs + 63) / 64), dim3(64), 0, s, bv);
  return hipGetLastError();
}

void job_phase_blocks(const Dims& d, int counts[PH_COUNT]) {
  counts[PH_GHOST] = (ghost_threads(d) + 255) / 256;
  counts[PH_SWEEP] = (int)sweep_blocks(d);
  counts[PH_UPDATE] = (int)xcd_grid(d.n1, d.n2, d.n3, d.utx, d.uty);
}
