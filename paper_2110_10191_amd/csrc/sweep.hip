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
// Courant step (one atomic max per block).
#include "kernels.h"

namespace {

template <int D, int RECON, typename T>
__global__ __launch_bounds__(256) void sweep_kernel(Dims d, const double* __restrict__ P,
                                                    const T* __restrict__ tab, T* __restrict__ F,
                                                    T gam, int lo1, int cnt1, int lo2, int cnt2,
                                                    int lo3, int cnt3, int tiles_x, int chunk,
                                                    unsigned long long* ctop) {
  const TileK t = xcd_tile_k(tiles_x, cnt3, chunk);
  const int i = lo1 + t.i0 + (int)threadIdx.x;
  const int j = lo2 + t.j0 + (int)threadIdx.y;
  const int k = lo3 + t.k;
  const bool active = t.valid && (i < lo1 + cnt1) && (j < lo2 + cnt2);
  double cmx = 0.0;
  if (active) {
    const int c = cell_of(d, k, j, i);
    const int st = (D == 1) ? 1 : ((D == 2) ? d.s2 : d.s3);
    T PL[NV], PR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double* q = P + v * d.sv + c;
      if (RECON == GRMHD_RECON_MC) {
        const T a = (T)q[-2 * st], b = (T)q[-st], e = (T)q[0], f = (T)q[st];
        PL[v] = b + T(0.5) * mc_slope(a, b, e);
        PR[v] = e - T(0.5) * mc_slope(b, e, f);
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
#pragma unroll
    for (int v = 0; v < NV; ++v) F[v * d.sv + c] = T(0.5) * (FL[v] + FR[v]) - T(0.5) * ct * (UR[v] - UL[v]);
    bool inner;
    if (D == 1) inner = (j >= 0 && j < d.n2 && k >= 0 && k < d.n3);
    else if (D == 2) inner = (i >= 0 && i < d.n1 && k >= 0 && k < d.n3);
    else inner = (i >= 0 && i < d.n1 && j >= 0 && j < d.n2);
    if (inner) {
      cmx = (double)ct;
      if (cmx != cmx) cmx = __builtin_inf();
    }
  }
  if (ctop) block_max_to(cmx, ctop + (D - 1));
}

template <int D, int RECON, typename T>
void launch_one(const Dims& d, const T* tab, double gam, const double* P, T* F, unsigned long long* ctop,
                hipStream_t s) {
  const int lo1 = (D == 1) ? 0 : -1, c1 = (D == 1) ? d.n1 + 1 : d.n1 + 2;
  const int lo2 = (D == 2) ? 0 : -1, c2 = (D == 2) ? d.n2 + 1 : d.n2 + 2;
  const int lo3 = (D == 3) ? 0 : -1, c3 = (D == 3) ? d.n3 + 1 : d.n3 + 2;
  int tiles_x, chunk;
  const unsigned nblk = xcd_grid(c1, c2, c3, &tiles_x, &chunk);
  hipLaunchKernelGGL((sweep_kernel<D, RECON, T>), dim3(nblk), dim3(TILE_X, TILE_Y, 1), 0, s, d, P, tab, F,
                     (T)gam, lo1, c1, lo2, c2, lo3, c3, tiles_x, chunk, ctop);
}

template <int RECON, typename T>
void launch_dir(int dir, const Dims& d, const T* cent, const T* f1, const T* f2, double gam,
                const double* P, T* F, unsigned long long* ctop, hipStream_t s) {
  if (dir == 1) launch_one<1, RECON, T>(d, f1, gam, P, F, ctop, s);
  else if (dir == 2) launch_one<2, RECON, T>(d, f2, gam, P, F, ctop, s);
  else launch_one<3, RECON, T>(d, cent, gam, P, F, ctop, s);
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
