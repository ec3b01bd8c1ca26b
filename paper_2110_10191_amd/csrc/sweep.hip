// Face fluxes of all three directions in one pass: reconstruct the primitives
// at the lower d-face of each zone (MC or WENO5), evaluate both face states
// (four-velocity, field four-vector, flux, conserved variables, fast-
// magnetosonic speeds) and combine them with the local Lax-Friedrichs flux
//   F = (F_L + F_R)/2 - ctop (U_R - U_L)/2,
//   ctop = max(max(0, c+_L, c+_R), max(0, -c-_L, -c-_R)).
// Functionality section: HARM updates conserved variables by finite volumes;
// the reconstruction and Riemann solver follow the HARM literature.
//
// Faces covered in direction d: 0..n_d along d, and -1..n_t in both
// transverse directions (the extra transverse layer feeds the Flux-CT EMFs).
// One thread per cell (i, j, k) with i, j, k in [-1, n] computes the faces of
// every direction whose range holds it, so a cell's primitives are read from
// HBM once for the three directions and one launch replaces three. A block
// first copies its tile of the x3 plane, with the reconstruction halo in x1
// and x2, into LDS (coalesced along x1); the x1 and x2 stencils then come
// from LDS and only the other planes of the x3 stencil from the state. The
// per-direction maximum of ctop over the faces with interior transverse index
// feeds the Courant step (one atomic max per block and direction); a face with
// a NaN speed counts as +inf there, which the step reports as a non-finite
// state. The face geometry comes from the face tables, or for Cartesian
// Kerr-Schild in FP64 from its closed form (the same bits as the table).
#include <atomic>
#include <type_traits>

#include "cks_geometry.h"
#include "kernels.h"

namespace {

// the block's x3 plane of primitives with the stencil halo in x1 and x2,
// [8][lh][lw] of T, cells (ib + li, jb + lj)
template <typename T>
struct PlaneTile {
  const T* lds;
  int lw, lh;    // row length and rows
  int li, lj;    // this thread's cell in the tile
  int plane;     // lw * lh
};

// halo of the reconstruction: zones below / above the cell (MC 2 / 1, WENO5 3 / 2)
template <int RECON>
constexpr int halo_lo() { return RECON == GRMHD_RECON_MC ? 2 : 3; }
template <int RECON>
constexpr int halo_hi() { return RECON == GRMHD_RECON_MC ? 1 : 2; }

// the face of direction D at the lower D-face of cell (k, j, i): store the
// flux (all but the face-normal field component, which Flux-CT replaces by
// zero and nothing reads) and return the signal speed for the Courant maximum
// (0 for a face with a transverse ghost index, +inf when its speeds are not
// finite)
// CKS: the face geometry of Cartesian Kerr-Schild computed in closed form
// (the values of the face table) instead of read
template <int D, int RECON, typename T, bool CKS>
__device__ inline double one_face(const Dims& d, const double* __restrict__ P, const PlaneTile<T>& pt,
                                  const T* __restrict__ tab, const CksBox& box, T* __restrict__ F, T gam, int i,
                                  int j, int k) {
  const int c = cell_of(d, k, j, i);
  T PL[NV], PR[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    // x1 and x2 stencils from the LDS tile, x3 from the state
    const T* ql = pt.lds + v * pt.plane + pt.lj * pt.lw + pt.li;
    const double* qg = P + v * d.sv + c;
    const int st = (D == 1) ? 1 : pt.lw;
    // the cell's own value from the LDS tile in every direction
    auto at = [&](int o) -> T { return (D == 3 && o != 0) ? (T)qg[o * d.s3] : ql[o * st]; };
    if (RECON == GRMHD_RECON_MC) {
      const T a = at(-2), bb = at(-1), e = at(0), f = at(1);
      PL[v] = bb + T(0.5) * mc_slope(a, bb, e);
      PR[v] = e - T(0.5) * mc_slope(bb, e, f);
    } else {
      const T x0 = at(-3), x1 = at(-2), x2 = at(-1), x3 = at(0), x4 = at(1), x5 = at(2);
      PL[v] = weno5_edge(x0, x1, x2, x3, x4);
      PR[v] = weno5_edge(x5, x4, x3, x2, x1);
    }
  }
  Geo<T> g;
  if constexpr (CKS) cks_face_geo(box, D, i, j, k, g);
  else load_face_geo(g, face_plane(tab, d, k), d.ts, tab_of(d, j, i));
  T FL[NV], UL[NV], cpL, cmL;
  {
    Fluid<T> f;
    fluid_state<T, true>(PL, g, gam, f);
    flux_of<D>(PL, f, g.gdet, FL);
    flux_of<0>(PL, f, g.gdet, UL);
    signal_speeds<D>(f, g, gam, cpL, cmL);
  }
  T FR[NV], UR[NV], cpR, cmR;
  {
    Fluid<T> f;
    fluid_state<T, true>(PR, g, gam, f);
    flux_of<D>(PR, f, g.gdet, FR);
    flux_of<0>(PR, f, g.gdet, UR);
    signal_speeds<D>(f, g, gam, cpR, cmR);
  }
  const T cmax = fmax(fmax(T(0), cpL), cpR);
  const T cmin = fmax(fmax(T(0), -cmL), -cmR);
  const T ct = fmax(cmax, cmin);
  T fv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) fv[v] = T(0.5) * (FL[v] + FR[v]) - T(0.5) * ct * (UR[v] - UL[v]);
  // no mass enters through an outflow boundary: the rest-mass flux through
  // the inner radial face is at most 0, through the outer one at least 0
  if (D == 1 && d.out_lo && i == 0) fv[0] = fmin(fv[0], T(0));
  if (D == 1 && d.out_hi && i == d.n1) fv[0] = fmax(fv[0], T(0));
#pragma unroll
  for (int v = 0; v < NV; ++v)
    if (v != 4 + D) F[v * d.sv + c] = fv[v];
  bool inner;
  if (D == 1) inner = (j >= 0 && j < d.n2 && k >= 0 && k < d.n3);
  else if (D == 2) inner = (i >= 0 && i < d.n1 && k >= 0 && k < d.n3);
  else inner = (i >= 0 && i < d.n1 && j >= 0 && j < d.n2);
  if (!inner) return 0.0;
  // fmax drops a NaN operand, so a face whose states are not finite would
  // report a finite (often zero) speed: any NaN speed makes it +inf, so the
  // Courant step sees the non-finite state
  const T chk = (cpL + cmL) + (cpR + cmR);
  return (chk == chk) ? (double)ct : __builtin_inf();
}

// b: block index within this job's grid of tiles over (n1+2) x (n2+2) x (n3+2)
// cells starting at (-1, -1, -1)
template <int RECON, typename T, bool CKS = false>
__device__ void sweep_body(const Dims& d, const double* __restrict__ P, const T* __restrict__ t1,
                           const T* __restrict__ t2, const T* __restrict__ t3, const CksBox& box, T* __restrict__ F1,
                           T* __restrict__ F2, T* __restrict__ F3, T gam, int b, unsigned long long* ctop) {
  const TileK t = xcd_tile_k(b, d.stx, d.sty, d.n1 + 2, d.n3 + 2);
  const int i = -1 + t.i0 + (int)threadIdx.x;
  const int j = -1 + t.j0 + (int)threadIdx.y;
  const int k = -1 + t.k;
  const bool ok = t.valid && i <= d.n1 && j <= d.n2;
  // stage this x3 plane of the tile and its x1 / x2 halo in LDS, once for the
  // block: cells [ib, ib + lw) x [jb, jb + lh), those inside the padded state
  // (cells outside it are never read: faces start at cell 0 and end at n)
  extern __shared__ __align__(16) unsigned char sweep_lds[];
  PlaneTile<T> pt;
  pt.lds = reinterpret_cast<const T*>(sweep_lds);
  pt.lw = d.stx + halo_lo<RECON>() + halo_hi<RECON>();
  pt.lh = d.sty + halo_lo<RECON>() + halo_hi<RECON>();
  pt.plane = pt.lw * pt.lh;
  pt.li = (int)threadIdx.x + halo_lo<RECON>();
  pt.lj = (int)threadIdx.y + halo_lo<RECON>();
  if (t.valid) {
    T* L = reinterpret_cast<T*>(sweep_lds);
    const int ib = -1 + t.i0 - halo_lo<RECON>(), jb = -1 + t.j0 - halo_lo<RECON>();
    const int nthr = d.stx * d.sty;
    for (int e = (int)threadIdx.y * d.stx + (int)threadIdx.x; e < pt.plane; e += nthr) {
      const int lj = e / pt.lw, li = e - lj * pt.lw;
      const int gi = ib + li, gj = jb + lj;
      if (gi >= -NG && gi < d.n1 + NG && gj >= -NG && gj < d.n2 + NG) {
        const int c = cell_of(d, k, gj, gi);
#pragma unroll
        for (int v = 0; v < NV; ++v) L[v * pt.plane + e] = (T)P[v * d.sv + c];
      }
    }
  }
  __syncthreads();
  double c1 = 0.0, c2 = 0.0, c3 = 0.0;
  if (ok && i >= 0) c1 = one_face<1, RECON, T, CKS>(d, P, pt, t1, box, F1, gam, i, j, k);
  if (ok && j >= 0) c2 = one_face<2, RECON, T, CKS>(d, P, pt, t2, box, F2, gam, i, j, k);
  if (ok && k >= 0) c3 = one_face<3, RECON, T, CKS>(d, P, pt, t3, box, F3, gam, i, j, k);
  if (ctop) block_max3_to(c1, c2, c3, ctop);
}

template <int RECON, typename T, bool CKS>
__global__ __launch_bounds__(512) void sweep_kernel(Dims d, const double* __restrict__ P, const T* __restrict__ t1,
                                                    const T* __restrict__ t2, const T* __restrict__ t3, CksBox box,
                                                    T* __restrict__ F1, T* __restrict__ F2, T* __restrict__ F3, T gam,
                                                    unsigned long long* ctop) {
  sweep_body<RECON, T, CKS>(d, P, t1, t2, t3, box, F1, F2, F3, gam, (int)blockIdx.x, ctop);
}

template <typename T>
struct FaceTables;
template <>
struct FaceTables<double> {
  __host__ __device__ static const double* f1(const Tables& t) { return t.f1; }
  __host__ __device__ static const double* f2(const Tables& t) { return t.f2; }
  __host__ __device__ static const double* f3(const Tables& t) { return t.f3; }
};
template <>
struct FaceTables<float> {
  __host__ __device__ static const float* f1(const Tables& t) { return t.f1f; }
  __host__ __device__ static const float* f2(const Tables& t) { return t.f2f; }
  __host__ __device__ static const float* f3(const Tables& t) { return t.f3f; }
};

// every job of a batch in one grid; predictor sweeps P, corrector sweeps P_h
template <int RECON, typename T>
__global__ __launch_bounds__(512) void sweep_batch_kernel(BatchView bv, int corrector, int want_ctop) {
  const int* offs = bv.offs + PH_SWEEP * (bv.njobs + 1);
  const int jb = batch_job(offs, bv.njobs, (int)blockIdx.x);
  const JobDesc& J = bv.jobs[jb];
  const CksBox none{};
  sweep_body<RECON, T>(J.d, global_ptr(corrector ? J.Ph : J.P), global_ptr(FaceTables<T>::f1(J.t)),
                       global_ptr(FaceTables<T>::f2(J.t)), global_ptr(FaceTables<T>::f3(J.t)), none,
                       global_ptr((T*)J.F[0]), global_ptr((T*)J.F[1]), global_ptr((T*)J.F[2]), (T)J.p.gam,
                       (int)blockIdx.x - offs[jb], want_ctop ? global_ptr(J.ctr->ctop) : nullptr);
}

template <int RECON, typename T>
size_t tile_bytes(int stx, int sty) {
  return (size_t)NV * (stx + halo_lo<RECON>() + halo_hi<RECON>()) * (sty + halo_lo<RECON>() + halo_hi<RECON>()) *
         sizeof(T);
}

// A kernel may use more dynamic LDS than the default 64 KiB only once the
// limit is raised for it; the largest limit set so far is kept per kernel.
template <auto KERNEL>
hipError_t allow_lds(size_t bytes) {
  static std::atomic<size_t> allowed{65536};
  if (bytes <= allowed.load()) return hipSuccess;
  const hipError_t e = hipFuncSetAttribute((const void*)KERNEL, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) {
    size_t cur = allowed.load();
    while (cur < bytes && !allowed.compare_exchange_weak(cur, bytes)) {
    }
  }
  return e;
}

template <int RECON, typename T, bool CKS>
hipError_t launch_geo(const Dims& d, const Tables& t, const CksBox& box, double gam, const double* P,
                      void* const* F, unsigned long long* ctop, hipStream_t s) {
  const unsigned nblk = sweep_blocks(d);
  const size_t lds = tile_bytes<RECON, T>(d.stx, d.sty);
  const hipError_t e = allow_lds<sweep_kernel<RECON, T, CKS>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((sweep_kernel<RECON, T, CKS>), dim3(nblk), dim3(d.stx, d.sty, 1), lds, s, d, P,
                     FaceTables<T>::f1(t), FaceTables<T>::f2(t), FaceTables<T>::f3(t), box, (T*)F[0], (T*)F[1],
                     (T*)F[2], (T)gam, ctop);
  return hipGetLastError();
}

// Cartesian Kerr-Schild in FP64 computes its face geometry instead of
// streaming the 3D face tables (most of the bytes the pass moved); the
// FP32 pass reads the float tables, cheaper than evaluating the metric in
// FP64; the other coordinates read their 2D tables
template <int RECON, typename T>
hipError_t launch_for(const grmhd_problem& p, const Dims& d, const Tables& t, const double* P, void* const* F,
                      unsigned long long* ctop, hipStream_t s) {
  if (std::is_same<T, double>::value && p.coords == GRMHD_KERR_CKS)
    return launch_geo<RECON, T, true>(d, t, cks_box(p), p.gam, P, F, ctop, s);
  return launch_geo<RECON, T, false>(d, t, CksBox{}, p.gam, P, F, ctop, s);
}

template <int RECON, typename T>
hipError_t launch_batch_for(const BatchView& bv, dim3 grd, dim3 blk, int c, int w, hipStream_t s) {
  const size_t lds = tile_bytes<RECON, T>(bv.stx, bv.sty);
  const hipError_t e = allow_lds<sweep_batch_kernel<RECON, T>>(lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((sweep_batch_kernel<RECON, T>), grd, blk, lds, s, bv, c, w);
  return hipGetLastError();
}

}  // namespace

unsigned sweep_blocks(const Dims& d) { return xcd_grid(d.n1 + 2, d.n2 + 2, d.n3 + 2, d.stx, d.sty); }

hipError_t launch_sweeps(const grmhd_problem& p, bool mixed, const Dims& d, const Tables& t, const double* P,
                         void* const* F, unsigned long long* ctop, hipStream_t s) {
  if (mixed) {
    if (p.recon == GRMHD_RECON_MC) return launch_for<GRMHD_RECON_MC, float>(p, d, t, P, F, ctop, s);
    return launch_for<GRMHD_RECON_WENO5, float>(p, d, t, P, F, ctop, s);
  }
  if (p.recon == GRMHD_RECON_MC) return launch_for<GRMHD_RECON_MC, double>(p, d, t, P, F, ctop, s);
  return launch_for<GRMHD_RECON_WENO5, double>(p, d, t, P, F, ctop, s);
}

hipError_t launch_batch_sweeps(const BatchView& bv, const int* totals, int recon, bool mixed, bool corrector,
                               bool want_ctop, hipStream_t s) {
  const dim3 blk(bv.stx, bv.sty, 1), grd(totals[PH_SWEEP]);
  const int c = corrector ? 1 : 0, w = want_ctop ? 1 : 0;
  if (mixed) {
    if (recon == GRMHD_RECON_MC) return launch_batch_for<GRMHD_RECON_MC, float>(bv, grd, blk, c, w, s);
    return launch_batch_for<GRMHD_RECON_WENO5, float>(bv, grd, blk, c, w, s);
  }
  if (recon == GRMHD_RECON_MC) return launch_batch_for<GRMHD_RECON_MC, double>(bv, grd, blk, c, w, s);
  return launch_batch_for<GRMHD_RECON_WENO5, double>(bv, grd, blk, c, w, s);
}
