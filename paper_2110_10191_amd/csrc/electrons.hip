// Electron heating (Implementation Notes: the dissipation is tracked and split
// between ions and electrons after Ressler et al. 2015, with the heating
// models of Kawazura et al. 2019, Werner et al. 2018, Rowan et al. 2017,
// Howes 2010 and Sharma et al. 2007). Two passes per substep around the fluid update:
//
//   scalar advection (after the sweeps, before the fluid update overwrites the
//   base state): for both entropies K (K_tot = P_gas / rho^gamma and
//   K_e = P_e / rho^gamma_e, gamma_e = 4/3)
//     U_K = sqrt(-g) rho_b u^t_b K_b - dt sum_d [F_K(+) - F_K(-)] / dx_d,
//     F_K = F_mass K*, K* the face value (the fluid's reconstruction) on the
//     upwind side of the mass flux; the mass flux through a polar axis is 0;
//
//   heating (after the fluid update, bounds and fixup): u <= 3 rho^gamma /
//   (gamma - 1) (P_gas / rho^gamma < 3); with D = sqrt(-g) rho u^t of the new
//   state, K_adv = U_K / D and K = (gamma - 1) u / rho^gamma,
//     K_e = K_e,adv + f_e (gamma_e - 1)/(gamma - 1) rho^(gamma - gamma_e) (K - K_tot,adv)
//   (the electrons receive the fraction f_e of the dissipated internal
//   energy), bounded to [0, rho^(gamma - gamma_e) K] (0 <= P_e <= P_gas), and
//   K_tot = K.
//
// f_e is a constant or a model of beta_i = P_i / (b^2/2), T_e/T_i = P_e / P_i
// (P_i = P_gas - P_e), sigma = b^2/rho and sigma_w = b^2 / (rho + u + P_gas):
//   Kawazura: Q_i/Q_e = 35 / (1 + (beta_i/15)^-1.4 exp(-0.1 T_e/T_i));
//   Werner:   f_e = (1 + sqrt((sigma/5) / (2 + sigma/5))) / 4;
//   Rowan:    f_e = exp(-max(1 - beta_i/beta_max, 0)^3.3 / (1 + 1.2 sigma_w^0.7)) / 2,
//             beta_max = 1/(4 sigma_w);
//   Howes:    theta = T_i/T_e, Q_i/Q_e = 0.92 (c2^2 + beta_i^x)/(c3^2 + beta_i^x)
//             sqrt(theta m_p/m_e) exp(-1/beta_i), x = 2 - 0.2 log10 theta,
//             c2 = 1.6/theta, c3 = 18 + 5 log10 theta for theta > 1,
//             c2 = 1.2/theta, c3 = 18 otherwise, beta_i^x capped at e^700;
//   Sharma:   Q_e/Q_i = sqrt(T_e/T_i) / 3, i.e. Q_i/Q_e = 3 sqrt(T_i/T_e);
// with f_e = 1 / (1 + Q_i/Q_e) where a ratio is given.
#include "kernels.h"

namespace {

constexpr double GAM_E = 4.0 / 3.0;
constexpr double KAPPA_MAX = 3.0;
constexpr double MP_ME = 1836.15267343;

// the two face values of a scalar at the lower face of the zone at q (stride st)
template <int RECON>
__device__ inline void scalar_faces(const double* q, int st, double& l, double& r) {
  if (RECON == GRMHD_RECON_MC) {
    const double a = q[-2 * st], b = q[-st], e = q[0], f = q[st];
    l = b + 0.5 * mc_slope(a, b, e);
    r = e - 0.5 * mc_slope(b, e, f);
  } else {
    const double x0 = q[-3 * st], x1 = q[-2 * st], x2 = q[-st], x3 = q[0], x4 = q[st], x5 = q[2 * st];
    l = weno5_edge(x0, x1, x2, x3, x4);
    r = weno5_edge(x5, x4, x3, x2, x1);
  }
}

// upwind flux of both scalars through the lower face (stride st) of cell c
template <int RECON>
__device__ inline void scalar_flux(const double* E, int sv, int c, int st, double m, double f[GRMHD_NSCALAR]) {
#pragma unroll
  for (int s = 0; s < GRMHD_NSCALAR; ++s) {
    double l, r;
    scalar_faces<RECON>(E + s * sv + c, st, l, r);
    f[s] = m * (m >= 0.0 ? l : r);
  }
}

// b: block index within this job's grid (the update tile, XCD-aware order)
template <typename TF, int RECON>
__device__ void scalar_advect_body(const Dims& d, const double* __restrict__ cent, const UpdateParams& up,
                                   const TF* __restrict__ F1, const TF* __restrict__ F2, const TF* __restrict__ F3,
                                   const double* __restrict__ Pb, const double* __restrict__ Eb,
                                   const double* __restrict__ Es, double* __restrict__ Uk, double dt, int b) {
  const TileK tk = xcd_tile_k(b, d.utx, d.uty, d.n1, d.n3);
  const int i = tk.i0 + (int)threadIdx.x;
  const int j = tk.j0 + (int)threadIdx.y;
  if (!tk.valid || i >= d.n1 || j >= d.n2) return;
  const int c = cell_of(d, tk.k, j, i);
  const bool pl = up.polar_lo && j == 0;
  const bool ph = up.polar_hi && j == d.n2 - 1;
  double fm[GRMHD_NSCALAR], fp[GRMHD_NSCALAR], div[GRMHD_NSCALAR];
  scalar_flux<RECON>(Es, d.sv, c, 1, (double)F1[c], fm);
  scalar_flux<RECON>(Es, d.sv, c + 1, 1, (double)F1[c + 1], fp);
#pragma unroll
  for (int s = 0; s < GRMHD_NSCALAR; ++s) div[s] = (fp[s] - fm[s]) * up.idx1;
  scalar_flux<RECON>(Es, d.sv, c, d.s2, pl ? 0.0 : (double)F2[c], fm);
  scalar_flux<RECON>(Es, d.sv, c + d.s2, d.s2, ph ? 0.0 : (double)F2[c + d.s2], fp);
#pragma unroll
  for (int s = 0; s < GRMHD_NSCALAR; ++s) div[s] += (fp[s] - fm[s]) * up.idx2;
  scalar_flux<RECON>(Es, d.sv, c, d.s3, (double)F3[c], fm);
  scalar_flux<RECON>(Es, d.sv, c + d.s3, d.s3, (double)F3[c + d.s3], fp);
#pragma unroll
  for (int s = 0; s < GRMHD_NSCALAR; ++s) div[s] += (fp[s] - fm[s]) * up.idx3;

  // rest-mass density of the base state: sqrt(-g) rho u^t, u^t = Gamma / alpha
  const int toff = tab_of(d, j, i);
  const double* ck = tab_plane(cent, d, tk.k);
  double gcov[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) gcov[m] = ck[(T_GCOV + m) * d.ts + toff];
  const double gdet = ck[T_GDET * d.ts + toff], alpha = ck[T_ALPHA * d.ts + toff];
  const double ut = sqrt(lorentz_sq(gcov, Pb[2 * d.sv + c], Pb[3 * d.sv + c], Pb[4 * d.sv + c])) / alpha;
  const double D = gdet * Pb[c] * ut;
#pragma unroll
  for (int s = 0; s < GRMHD_NSCALAR; ++s) Uk[s * d.sv + c] = D * Eb[s * d.sv + c] - dt * div[s];
}

template <typename TF, int RECON>
__global__ __launch_bounds__(256) void scalar_advect_kernel(Dims d, const double* __restrict__ cent, UpdateParams up,
                                                            const TF* __restrict__ F1, const TF* __restrict__ F2,
                                                            const TF* __restrict__ F3, const double* __restrict__ Pb,
                                                            const double* __restrict__ Eb, const double* __restrict__ Es,
                                                            double* __restrict__ Uk, double dt,
                                                            const double* __restrict__ dt_dev, double dt_scale) {
  if (dt_dev) dt = dt_scale * *dt_dev;
  scalar_advect_body<TF, RECON>(d, cent, up, F1, F2, F3, Pb, Eb, Es, Uk, dt, (int)blockIdx.x);
}

// every job with entropies in one grid: predictor (E -> U_K, base P), corrector
// (E_h fluxes, base E and P)
template <typename TF, int RECON>
__global__ __launch_bounds__(256) void scalar_advect_batch_kernel(BatchView bv, int corrector) {
  const int* offs = bv.offs + PH_UPDATE * (bv.njobs + 1);
  const int jb = batch_job(offs, bv.njobs, (int)blockIdx.x);
  const JobDesc& J = bv.jobs[jb];
  if (!J.E) return;
  const double dt = corrector ? *J.dt : 0.5 * *J.dt;
  scalar_advect_body<TF, RECON>(J.d, global_ptr(J.t.cent), J.up, global_ptr((const TF*)J.F[0]),
                                global_ptr((const TF*)J.F[1]), global_ptr((const TF*)J.F[2]), global_ptr(J.P),
                                global_ptr(J.E), global_ptr(corrector ? J.Eh : J.E), global_ptr(J.Uk), dt,
                                (int)blockIdx.x - offs[jb]);
}

__device__ double heating_fraction(int model, double fel, double rho, double u, double kel, double bsq, double gam) {
  if (model == GRMHD_HEAT_CONSTANT) return fel;
  const double pg = (gam - 1.0) * u;
  const double pe = kel * pow(rho, GAM_E);
  const double pi = fmax(pg - pe, 1e-30 * pg + 1e-300);
  const double pb = 0.5 * bsq + 1e-300;
  const double beta = pi / pb;
  if (model == GRMHD_HEAT_KAWAZURA) {
    const double qi_qe = 35.0 / (1.0 + pow(beta / 15.0, -1.4) * exp(-0.1 * (pe / pi)));
    return 1.0 / (1.0 + qi_qe);
  }
  if (model == GRMHD_HEAT_WERNER) {
    const double s5 = bsq / rho / 5.0;
    return 0.25 * (1.0 + sqrt(s5 / (2.0 + s5)));
  }
  if (model == GRMHD_HEAT_ROWAN) {
    const double sw = bsq / (rho + u + pg);
    const double bmax = 1.0 / (4.0 * sw + 1e-300);
    const double x = fmax(1.0 - beta / bmax, 0.0);
    return 0.5 * exp(-pow(x, 3.3) / (1.0 + 1.2 * pow(sw, 0.7)));
  }
  if (model == GRMHD_HEAT_SHARMA) return 1.0 / (1.0 + 3.0 * sqrt(pi / fmax(pe, 1e-300)));
  // Howes
  const double theta = pi / fmax(pe, 1e-300);
  const double lt = log10(theta);
  const double c2 = (theta > 1.0 ? 1.6 : 1.2) / theta;
  const double c3 = theta > 1.0 ? 18.0 + 5.0 * lt : 18.0;
  const double x = 2.0 - 0.2 * lt;
  const double bx = exp(fmin(x * log(beta), 700.0));
  const double qi_qe = 0.92 * (c2 * c2 + bx) / (c3 * c3 + bx) * sqrt(MP_ME * theta) * exp(-1.0 / beta);
  return 1.0 / (1.0 + qi_qe);
}

// b: block index within this job's grid
__device__ void electron_heat_body(const Dims& d, const double* __restrict__ cent, double gam, double* __restrict__ P,
                                   const double* __restrict__ Uk, double* __restrict__ E, int model, double fel,
                                   unsigned* bad, int b) {
  const TileK tk = xcd_tile_k(b, d.utx, d.uty, d.n1, d.n3);
  const int i = tk.i0 + (int)threadIdx.x;
  const int j = tk.j0 + (int)threadIdx.y;
  if (!tk.valid || i >= d.n1 || j >= d.n2) return;
  const int c = cell_of(d, tk.k, j, i);
  double p[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) p[v] = P[v * d.sv + c];
  const double rho = p[0];
  const double rg = pow(rho, gam);
  const double umax = KAPPA_MAX * rg / (gam - 1.0);
  if (p[1] > umax) {
    p[1] = umax;
    P[d.sv + c] = umax;
  }
  Geo<double> g;
  load_geo(g, tab_plane(cent, d, tk.k), d.ts, tab_of(d, j, i));
  Fluid<double> f;
  fluid_state(p, g, gam, f);
  const double D = g.gdet * rho * f.ucon[0];
  const double ktot_adv = Uk[c] / D, kel_adv = Uk[d.sv + c] / D;
  const double ktot = (gam - 1.0) * p[1] / rg;
  const double fe = heating_fraction(model, fel, rho, p[1], kel_adv, f.bsq, gam);
  const double scale = pow(rho, gam - GAM_E);
  double kel = kel_adv + fe * (GAM_E - 1.0) / (gam - 1.0) * scale * (ktot - ktot_adv);
  kel = fmin(fmax(kel, 0.0), scale * ktot);
  E[c] = ktot;
  E[d.sv + c] = kel;
  if (!(isfinite(ktot) && isfinite(kel))) atomicAdd(bad, 1u);
}

__global__ __launch_bounds__(256) void electron_heat_kernel(Dims d, const double* __restrict__ cent, double gam,
                                                            double* __restrict__ P, const double* __restrict__ Uk,
                                                            double* __restrict__ E, int model, double fel,
                                                            Counters* ctr) {
  electron_heat_body(d, cent, gam, P, Uk, E, model, fel, &ctr->bad, (int)blockIdx.x);
}

// predictor: heats P_h into E_h; corrector: P into E
__global__ __launch_bounds__(256) void electron_heat_batch_kernel(BatchView bv, int corrector) {
  const int* offs = bv.offs + PH_UPDATE * (bv.njobs + 1);
  const int jb = batch_job(offs, bv.njobs, (int)blockIdx.x);
  const JobDesc& J = bv.jobs[jb];
  if (!J.E) return;
  electron_heat_body(J.d, global_ptr(J.t.cent), J.p.gam, global_ptr(corrector ? J.P : J.Ph), global_ptr(J.Uk),
                     global_ptr(corrector ? J.E : J.Eh), J.heat_model, J.fel, global_ptr(&J.ctr->bad),
                     (int)blockIdx.x - offs[jb]);
}

template <typename TF>
void advect_for(int recon, const Dims& d, const Tables& t, const UpdateParams& up, const void* F1, const void* F2,
                const void* F3, const double* Pb, const double* Eb, const double* Es, double* Uk, double dt,
                const double* dt_dev, double dt_scale, hipStream_t s) {
  const dim3 grid(xcd_grid(d.n1, d.n2, d.n3, d.utx, d.uty)), block(d.utx, d.uty, 1);
  const TF *f1 = (const TF*)F1, *f2 = (const TF*)F2, *f3 = (const TF*)F3;
  if (recon == GRMHD_RECON_MC)
    hipLaunchKernelGGL((scalar_advect_kernel<TF, GRMHD_RECON_MC>), grid, block, 0, s, d, t.cent, up, f1, f2, f3, Pb,
                       Eb, Es, Uk, dt, dt_dev, dt_scale);
  else
    hipLaunchKernelGGL((scalar_advect_kernel<TF, GRMHD_RECON_WENO5>), grid, block, 0, s, d, t.cent, up, f1, f2, f3,
                       Pb, Eb, Es, Uk, dt, dt_dev, dt_scale);
}

}  // namespace

hipError_t launch_scalar_advect(bool mixed, int recon, const Dims& d, const Tables& t, const UpdateParams& up,
                                const void* F1, const void* F2, const void* F3, const double* Pb, const double* Eb,
                                const double* Es, double* Uk, double dt, const double* dt_dev, double dt_scale,
                                hipStream_t s) {
  if (mixed) advect_for<float>(recon, d, t, up, F1, F2, F3, Pb, Eb, Es, Uk, dt, dt_dev, dt_scale, s);
  else advect_for<double>(recon, d, t, up, F1, F2, F3, Pb, Eb, Es, Uk, dt, dt_dev, dt_scale, s);
  return hipGetLastError();
}

hipError_t launch_batch_electrons(const BatchView& bv, const int* totals, bool mixed, int recon, bool corrector,
                                  int which, hipStream_t s) {
  if (which == 1) return launch_batch_scalar_ghosts(bv, totals, corrector, s);
  const dim3 grid(totals[PH_UPDATE]), block(bv.utx, bv.uty, 1);
  const int c = corrector ? 1 : 0;
  if (which == 2) {
    if (mixed) {
      if (recon == GRMHD_RECON_MC) hipLaunchKernelGGL((scalar_advect_batch_kernel<float, GRMHD_RECON_MC>), grid, block, 0, s, bv, c);
      else hipLaunchKernelGGL((scalar_advect_batch_kernel<float, GRMHD_RECON_WENO5>), grid, block, 0, s, bv, c);
    } else {
      if (recon == GRMHD_RECON_MC) hipLaunchKernelGGL((scalar_advect_batch_kernel<double, GRMHD_RECON_MC>), grid, block, 0, s, bv, c);
      else hipLaunchKernelGGL((scalar_advect_batch_kernel<double, GRMHD_RECON_WENO5>), grid, block, 0, s, bv, c);
    }
  } else {
    hipLaunchKernelGGL(electron_heat_batch_kernel, grid, block, 0, s, bv, c);
  }
  return hipGetLastError();
}

hipError_t launch_electron_heat(const Dims& d, const Tables& t, double gam, double* P, const double* Uk, double* E,
                                int model, double fel, Counters* ctr, hipStream_t s) {
  const dim3 grid(xcd_grid(d.n1, d.n2, d.n3, d.utx, d.uty)), block(d.utx, d.uty, 1);
  hipLaunchKernelGGL(electron_heat_kernel, grid, block, 0, s, d, t.cent, gam, P, Uk, E, model, fel, ctr);
  return hipGetLastError();
}
