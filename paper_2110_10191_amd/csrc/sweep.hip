// Face fluxes, one kernel per direction: reconstruct the primitives at the
// lower d-face of each zone (MC or WENO5), evaluate both face states (four-
// velocity, field four-vector, flux, conserved variables, fast-magnetosonic
// speeds) and combine them with the local Lax-Friedrichs flux
//   F = (F_L + F_R)/2 - ctop (U_R - U_L)/2,
//   ctop = max(max(0, c+_L, c+_R), max(0, -c-_L, -c-_R)).
// Functionality section: HARM is a conservative finite-volume scheme; the
// reconstruction and Riemann solver follow the HARM literature.
//
// Faces covered: 0..n_d along d, and -1..n_t in both transverse directions
// (the extra transverse layer feeds the Flux-CT EMFs). The per-direction
// maximum of ctop over the faces with interior transverse index feeds the
// Courant step (one atomic max per block); a face with a NaN speed counts as
// +inf there, which the step reports as a non-finite state.
#include "kernels.h"

namespace {

template <int D>
struct FaceRange {
  int lo1, c1, lo2, c2, lo3, c3;
  __host__ __device__ explicit FaceRange(const Dims& d)
      : lo1(D == 1 ? 0 : -1), c1(D == 1 ? d.n1 + 1 : d.n1 + 2), lo2(D == 2 ? 0 : -1),
        c2(D == 2 ? d.n2 + 1 : d.n2 + 2), lo3(D == 3 ? 0 : -1), c3(D == 3 ? d.n3 + 1 : d.n3 + 2) {}
};

// b: block index within this job's grid
template <int D, int RECON, typename T>
__device__ void sweep_body(const Dims& d, const double* __restrict__ P, const T* __restrict__ tab,
                           T* __restrict__ F, T gam, int b, unsigned long long* ctop) {
  const FaceRange<D> fr(d);
  const TileK t = xcd_tile_k(b, d.stx, d.sty, fr.c1, fr.c3);
  const int i = fr.lo1 + t.i0 + (int)threadIdx.x;
  const int j = fr.lo2 + t.j0 + (int)threadIdx.y;
  const int k = fr.lo3 + t.k;
  const bool active = t.valid && (i < fr.lo1 + fr.c1) && (j < fr.lo2 + fr.c2);
  double cmx = 0.0;
  if (active) {
    const int c = cell_of(d, k, j, i);
    const int st = (D == 1) ? 1 : ((D == 2) ? d.s2 : d.s3);
    T PL[NV], PR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double* q = P + v * d.sv + c;
      if (RECON == GRMHD_RECON_MC) {
        const T a = (T)q[-2 * st], bb = (T)q[-st], e = (T)q[0], f = (T)q[st];
        PL[v] = bb + T(0.5) * mc_slope(a, bb, e);
        PR[v] = e - T(0.5) * mc_slope(bb, e, f);
      } else {
        const T x0 = (T)q[-3 * st], x1 = (T)q[-2 * st], x2 = (T)q[-st], x3 = (T)q[0],
                x4 = (T)q[st], x5 = (T)q[2 * st];
        PL[v] = weno5_edge(x0, x1, x2, x3, x4);
        PR[v] = weno5_edge(x5, x4, x3, x2, x1);
      }
    }
    Geo<T> g;
    load_geo(g, tab, d.ts, tab_of(d, j, i));
    T FL[NV], UL[NV], cpL, cmL;
    {
      Fluid<T> f;
      fluid_state(PL, g, gam, f);
      flux_of<D>(PL, f, g.gdet, FL);
      flux_of<0>(PL, f, g.gdet, UL);
      signal_speeds<D>(f, g, gam, cpL, cmL);
    }
    T FR[NV], UR[NV], cpR, cmR;
    {
      Fluid<T> f;
      fluid_state(PR, g, gam, f);
      flux_of<D>(PR, f, g.gdet, FR);
      flux_of<0>(PR, f, g.gdet, UR);
      signal_speeds<D>(f, g, gam, cpR, cmR);
    }
    const T cmax = fmax(fmax(T(0), cpL), cpR);
    const T cmin = fmax(fmax(T(0), -cmL), -cmR);
    const T ct = fmax(cmax, cmin);
    // the flux of the face-normal field component (v = 4 + D) is not stored:
    // Flux-CT replaces it by zero, and nothing else reads it
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (v != 4 + D) F[v * d.sv + c] = T(0.5) * (FL[v] + FR[v]) - T(0.5) * ct * (UR[v] - UL[v]);
    bool inner;
    if (D == 1) inner = (j >= 0 && j < d.n2 && k >= 0 && k < d.n3);
    else if (D == 2) inner = (i >= 0 && i < d.n1 && k >= 0 && k < d.n3);
    else inner = (i >= 0 && i < d.n1 && j >= 0 && j < d.n2);
    if (inner) {
      // fmax drops a NaN operand, so a face whose states are not finite would
      // report a finite (often zero) speed: any NaN speed makes it +inf, so
      // the Courant step sees the non-finite state
      const T chk = (cpL + cmL) + (cpR + cmR);
      cmx = (chk == chk) ? (double)ct : __builtin_inf();
    }
  }
  if (ctop) block_max_to(cmx, ctop + (D - 1));
}

template <int D, int RECON, typename T>
__global__ __launch_bounds__(512) void sweep_kernel(Dims d, const double* __restrict__ P, const T* __restrict__ tab,
                                                    T* __restrict__ F, T gam, unsigned long long* ctop) {
  sweep_body<D, RECON, T>(d, P, tab, F, gam, (int)blockIdx.x, ctop);
}

template <typename T>
__device__ inline const T* face_table(const Tables& t, int dir);
template <>
__device__ inline const double* face_table<double>(const Tables& t, int dir) {
  return dir == 1 ? t.f1 : (dir == 2 ? t.f2 : t.cent);
}
template <>
__device__ inline const float* face_table<float>(const Tables& t, int dir) {
  return dir == 1 ? t.f1f : (dir == 2 ? t.f2f : t.centf);
}

// every job of a batch in one grid; predictor sweeps P, corrector sweeps P_h
template <int D, int RECON, typename T>
__global__ __launch_bounds__(512) void sweep_batch_kernel(BatchView bv, int corrector, int want_ctop) {
  const int* offs = bv.offs + (PH_SWEEP1 + D - 1) * (bv.njobs + 1);
  const int jb = batch_job(offs, bv.njobs, (int)blockIdx.x);
  const JobDesc& J = bv.jobs[jb];
  sweep_body<D, RECON, T>(J.d, global_ptr(corrector ? J.Ph : J.P), global_ptr(face_table<T>(J.t, D)),
                          global_ptr((T*)J.F[D - 1]), (T)J.p.gam, (int)blockIdx.x - offs[jb],
                          want_ctop ? global_ptr(J.ctr->ctop) : nullptr);
}

template <int D, int RECON, typename T>
void launch_one(const Dims& d, const T* tab, double gam, const double* P, T* F, unsigned long long* ctop,
                hipStream_t s) {
  const FaceRange<D> fr(d);
  const unsigned nblk = xcd_grid(fr.c1, fr.c2, fr.c3, d.stx, d.sty);
  hipLaunchKernelGGL((sweep_kernel<D, RECON, T>), dim3(nblk), dim3(d.stx, d.sty, 1), 0, s, d, P, tab, F,
                     (T)gam, ctop);
}

template <int RECON, typename T>
void launch_dir(int dir, const Dims& d, const T* cent, const T* f1, const T* f2, double gam,
                const double* P, T* F, unsigned long long* ctop, hipStream_t s) {
  if (dir == 1) launch_one<1, RECON, T>(d, f1, gam, P, F, ctop, s);
  else if (dir == 2) launch_one<2, RECON, T>(d, f2, gam, P, F, ctop, s);
  else launch_one<3, RECON, T>(d, cent, gam, P, F, ctop, s);
}

// dir 1..3: that direction only; 0: all three
template <int RECON, typename T>
void launch_batch_dirs(const BatchView& bv, const int* totals, bool corrector, bool want_ctop, int dir,
                       hipStream_t s) {
  const dim3 blk(bv.stx, bv.sty, 1);
  const int c = corrector ? 1 : 0, w = want_ctop ? 1 : 0;
  if (dir == 0 || dir == 1)
    hipLaunchKernelGGL((sweep_batch_kernel<1, RECON, T>), dim3(totals[PH_SWEEP1]), blk, 0, s, bv, c, w);
  if (dir == 0 || dir == 2)
    hipLaunchKernelGGL((sweep_batch_kernel<2, RECON, T>), dim3(totals[PH_SWEEP2]), blk, 0, s, bv, c, w);
  if (dir == 0 || dir == 3)
    hipLaunchKernelGGL((sweep_batch_kernel<3, RECON, T>), dim3(totals[PH_SWEEP3]), blk, 0, s, bv, c, w);
}

}  // namespace

hipError_t launch_sweep(int dir, int recon, bool mixed, const Dims& d, const Tables& t, double gam,
                        const double* P, void* F, unsigned long long* ctop, hipStream_t s) {
  if (mixed) {
    if (recon == GRMHD_RECON_MC)
      launch_dir<GRMHD_RECON_MC, float>(dir, d, t.centf, t.f1f, t.f2f, gam, P, (float*)F, ctop, s);
    else
      launch_dir<GRMHD_RECON_WENO5, float>(dir, d, t.centf, t.f1f, t.f2f, gam, P, (float*)F, ctop, s);
  } else {
    if (recon == GRMHD_RECON_MC)
      launch_dir<GRMHD_RECON_MC, double>(dir, d, t.cent, t.f1, t.f2, gam, P, (double*)F, ctop, s);
    else
      launch_dir<GRMHD_RECON_WENO5, double>(dir, d, t.cent, t.f1, t.f2, gam, P, (double*)F, ctop, s);
  }
  return hipGetLastError();
}

hipError_t launch_batch_sweeps(const BatchView& bv, const int* totals, int recon, bool mixed, bool corrector,
                               bool want_ctop, int dir, hipStream_t s) {
  if (mixed) {
    if (recon == GRMHD_RECON_MC) launch_batch_dirs<GRMHD_RECON_MC, float>(bv, totals, corrector, want_ctop, dir, s);
    else launch_batch_dirs<GRMHD_RECON_WENO5, float>(bv, totals, corrector, want_ctop, dir, s);
  } else {
    if (recon == GRMHD_RECON_MC) launch_batch_dirs<GRMHD_RECON_MC, double>(bv, totals, corrector, want_ctop, dir, s);
    else launch_batch_dirs<GRMHD_RECON_WENO5, double>(bv, totals, corrector, want_ctop, dir, s);
  }
  return hipGetLastError();
}
