// Zone update: Flux-CT, flux divergence, geometric source, 1D_W inversion and
// bounds, fused in one kernel per substep; the fixup of failed zones; and the
// pointwise prim->cons / cons->prim calls.
//
//   U* = U(P_base) + dt (-sum_d [F_d(+) - F_d(-)]/dx_d + S(P_s)),
//   S_nu = sqrt(-g) T^k_l Gamma^l_{nu k}                       (energy, momenta)
//   P_out = invert(U*; guess P_s), then the bounds, then the fixup.
//
// Flux-CT (Implementation Notes, after Toth 2000): the B fluxes through each
// face are replaced by the mean of the two edge EMFs bounding it, each EMF
// being the mean of the four face fluxes around its edge; that keeps the
// corner divergence of sqrt(-g) B unchanged. On polar axes the axis EMFs and
// the hydrodynamic x2 fluxes through the axis are zero.
//
// 1D_W (Implementation Notes, after Noble et al. 2006): Newton on W' = W - D for
// the root of the energy equation, with v^2(W) and p(W) written so nothing
// cancels at small u/rho or small v; converged once |dW'| <= 1e-8 W, then two
// more steps; at most 50 steps; v^2 clamped to [0, 1 - 1e-12] while iterating
// (with the clamp's zero derivative). Failure: no convergence, W <= 0,
// v^2 >= 1 - 1e-12 or non-finite; a failed zone keeps the guess's hydro
// primitives and is flagged for the fixup.
//
// Bounds (Implementation Notes): Gamma <= gamma_max by rescaling u~; then
// rho >= max(rho_fl k, b^2/sigma_max); u >= max(u_fl k^gamma, beta_min b^2/(2(gamma-1)));
// rho >= u/uorho_max; k = 1/(r^2 (1 + r/10)).
#include <type_traits>

#include "cks_geometry.h"
#include "kernels.h"

namespace {

constexpr double INV_TOL = 1e-8;
constexpr int INV_EXTRA = 2;
constexpr int INV_MAXIT = 50;
constexpr double V2MAX = 1.0 - 1e-12;

__device__ bool invert_1dw(const double* U, const double* guess, const Geo<double>& g, double gam,
                           double* P) {
  const double igd = 1.0 / g.gdet;
  const double a = g.alpha;
  const double ut0 = U[0] * igd, ut1 = U[1] * igd;
  const double D = a * ut0;
  const double Q1 = a * (U[2] * igd), Q2 = a * (U[3] * igd), Q3 = a * (U[4] * igd);
  const double Bu1 = U[5] * igd, Bu2 = U[6] * igd, Bu3 = U[7] * igd;
  const double B1 = a * Bu1, B2 = a * Bu2, B3 = a * Bu3;
  const double qn_d = ut1 + (a - 1.0) * ut0 - a * (g.gcon[1] * Q1 + g.gcon[2] * Q2 + g.gcon[3] * Q3);
  const double a2 = a * a;
  // spatial metric gamma^ij = g^ij + alpha^2 g^ti g^tj
  const double h11 = g.gcon[4] + a2 * g.gcon[1] * g.gcon[1];
  const double h12 = g.gcon[5] + a2 * g.gcon[1] * g.gcon[2];
  const double h13 = g.gcon[6] + a2 * g.gcon[1] * g.gcon[3];
  const double h22 = g.gcon[7] + a2 * g.gcon[2] * g.gcon[2];
  const double h23 = g.gcon[8] + a2 * g.gcon[2] * g.gcon[3];
  const double h33 = g.gcon[9] + a2 * g.gcon[3] * g.gcon[3];
  const double qt1 = h11 * Q1 + h12 * Q2 + h13 * Q3;
  const double qt2 = h12 * Q1 + h22 * Q2 + h23 * Q3;
  const double qt3 = h13 * Q1 + h23 * Q2 + h33 * Q3;
  const double qtsq = Q1 * qt1 + Q2 * qt2 + Q3 * qt3;
  const double qdb = Q1 * B1 + Q2 * B2 + Q3 * B3;
  const double qdb2 = qdb * qdb;
  const double bsq = g.gcov[4] * B1 * B1 + g.gcov[7] * B2 * B2 + g.gcov[9] * B3 * B3 +
                     2.0 * (g.gcov[5] * B1 * B2 + g.gcov[6] * B1 * B3 + g.gcov[8] * B2 * B3);
  const double gf = (gam - 1.0) / gam;

  double x = (guess[0] + gam * guess[1]) * lorentz_sq(g.gcov, guess[2], guess[3], guess[4]) - D;
  int extra = -1;
  for (int it = 0; it < INV_MAXIT && extra < INV_EXTRA; ++it) {
    // three divisions per iteration: 1/(W bw) gives 1/W and 1/bw,
    // 1/(s (1 + s)) gives 1/s and 1/(1 + s), and the Newton quotient
    const double W = x + D;
    const double W2 = W * W, bw = bsq + W;
    const double rwb = 1.0 / (W * bw);
    const double iW = bw * rwb, ibw = W * rwb;
    const double iW2 = iW * iW, ibw2 = ibw * ibw;
    const double v2raw = (qtsq * W2 + qdb2 * (bsq + 2.0 * W)) * (ibw2 * iW2);
    const double v2 = fmin(fmax(v2raw, 0.0), V2MAX);
    const double s = sqrt(1.0 - v2);
    const double rs = 1.0 / (s * (1.0 + s));
    const double is = (1.0 + s) * rs, i1s = s * rs;
    const double wmr = x * (1.0 - v2) - D * s * v2 * i1s;
    const double f = qn_d + x - gf * wmr + 0.5 * bsq * (1.0 + v2) - 0.5 * qdb2 * iW2;
    double dv2 = -2.0 * (qtsq * W2 * W + qdb2 * (3.0 * W2 + 3.0 * W * bsq + bsq * bsq)) * (ibw2 * ibw * iW2 * iW);
    if (v2raw > V2MAX || v2raw < 0.0) dv2 = 0.0;
    const double dp = gf * ((1.0 - v2) + (-W + 0.5 * D * is) * dv2);
    const double df = 1.0 - dp + 0.5 * bsq * dv2 + qdb2 * (iW2 * iW);
    const double dx = -f / df;
    double xn = x + dx;
    if (xn + D <= 0.0) xn = 0.5 * (x + D) - D;
    x = xn;
    if (extra < 0) {
      if (fabs(dx) <= INV_TOL * fabs(x + D)) extra = 0;
    } else {
      ++extra;
    }
  }
  const double W = x + D;
  const double bw = bsq + W;
  const double v2 = (qtsq * W * W + qdb2 * (bsq + 2.0 * W)) / (bw * bw * W * W);
  bool failed = (extra < 0) || !(W > 0.0) || !(v2 < V2MAX) || !isfinite(v2) || !isfinite(W);
  const double v2c = fmin(fmax(v2, 0.0), V2MAX);
  const double s = sqrt(1.0 - v2c);
  const double lor = 1.0 / s;
  P[0] = D * s;
  P[1] = (x * (1.0 - v2c) - D * s * v2c / (1.0 + s)) / gam;
  const double fac = lor / bw, qw = qdb / W;
  P[2] = fac * (qt1 + qw * B1);
  P[3] = fac * (qt2 + qw * B2);
  P[4] = fac * (qt3 + qw * B3);
  P[5] = Bu1;
  P[6] = Bu2;
  P[7] = Bu3;
  for (int v = 0; v < 5; ++v) failed = failed || !isfinite(P[v]);
  if (failed)
    for (int v = 0; v < 5; ++v) P[v] = guess[v];
  return failed;
}

__device__ void apply_floors(double* P, const Geo<double>& g, double rfl, double ufl, const UpdateParams& up) {
  const double lor2 = lorentz_sq(g.gcov, P[2], P[3], P[4]);
  const double gm2 = up.gamma_max * up.gamma_max;
  if (lor2 > gm2) {
    const double sc = sqrt((gm2 - 1.0) / (lor2 - 1.0));
    P[2] *= sc;
    P[3] *= sc;
    P[4] *= sc;
  }
  Fluid<double> f;
  fluid_state(P, g, up.gam, f);
  const double bsq = f.bsq;
  double rho = fmax(fmax(P[0], rfl), bsq / up.sigma_max);
  const double u = fmax(fmax(P[1], ufl), up.beta_min * bsq / (2.0 * (up.gam - 1.0)));
  rho = fmax(rho, u / up.uorho_max);
  P[0] = rho;
  P[1] = u;
}

template <typename TF>
struct FluxView {
  const TF* F;
  int sv;
  __device__ double at(int v, int c) const { return (double)F[v * sv + c]; }
  __device__ TF raw(int v, int c) const { return F[v * sv + c]; }
};

// b: block index within this job's grid (the update tile d.utx x d.uty, XCD-aware order)
// CKS: the centre metric of Cartesian Kerr-Schild computed in closed form
// (the values of the centre table) instead of read; the connection and the
// floor scales still come from the table
template <typename TF, bool EARLY_PS = false, bool CKS = false>
__device__ void update_body(const Dims& d, const double* __restrict__ cent, const CksBox& box, const UpdateParams& up,
                            const TF* __restrict__ F1p, const TF* __restrict__ F2p, const TF* __restrict__ F3p,
                            const double* Pb, const double* __restrict__ Ps, double* Pout,
                            int8_t* __restrict__ flags, double dt, Counters* ctr, int b) {
  const TileK tk = xcd_tile_k(b, d.utx, d.uty, d.n1, d.n3);
  const int i = tk.i0 + threadIdx.x;
  const int j = tk.j0 + threadIdx.y;
  const int k = tk.k;
  int failed = 0;
  if (tk.valid && i < d.n1 && j < d.n2) {
    const int c = cell_of(d, k, j, i);
    const FluxView<TF> F1{F1p, d.sv}, F2{F2p, d.sv}, F3{F3p, d.sv};
    const int s1 = 1, s2 = d.s2, s3 = d.s3;
    const bool pl = up.polar_lo && j == 0;
    const bool ph = up.polar_hi && j == d.n2 - 1;

    double ps[NV];
    if (EARLY_PS) {
#pragma unroll
      for (int v = 0; v < NV; ++v) ps[v] = Ps[v * d.sv + c];
    }
    double rhs[NV];
    // hydrodynamic flux divergence
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double f2m = pl ? 0.0 : F2.at(v, c);
      const double f2p = ph ? 0.0 : F2.at(v, c + s2);
      rhs[v] = -((F1.at(v, c + s1) - F1.at(v, c)) * up.idx1 + (f2p - f2m) * up.idx2 +
                 (F3.at(v, c + s3) - F3.at(v, c)) * up.idx3);
    }
    // Flux-CT: edge EMFs (in the flux precision)
    const TF q = TF(0.25), h = TF(0.5);
    // emf3 at edge (ii-1/2, jj-1/2, k), for ii in {i, i+1}, jj in {j, j+1}
    auto e3 = [&](int di, int dj) -> TF {
      const int jj = j + dj;
      if ((up.polar_lo && jj == 0) || (up.polar_hi && jj == d.n2)) return TF(0);
      const int cc = c + di * s1 + dj * s2;
      return q * (F1.raw(6, cc) + F1.raw(6, cc - s2) - F2.raw(5, cc) - F2.raw(5, cc - s1));
    };
    // emf1 at edge (i, jj-1/2, kk-1/2)
    auto e1 = [&](int dj, int dk) -> TF {
      const int jj = j + dj;
      if ((up.polar_lo && jj == 0) || (up.polar_hi && jj == d.n2)) return TF(0);
      const int cc = c + dj * s2 + dk * s3;
      return q * (F2.raw(7, cc) + F2.raw(7, cc - s3) - F3.raw(6, cc) - F3.raw(6, cc - s2));
    };
    // emf2 at edge (ii-1/2, j, kk-1/2)
    auto e2 = [&](int di, int dk) -> TF {
      const int cc = c + di * s1 + dk * s3;
      return q * (F3.raw(5, cc) + F3.raw(5, cc - s1) - F1.raw(7, cc) - F1.raw(7, cc - s3));
    };
    {
      const TF e3_00 = e3(0, 0), e3_10 = e3(1, 0), e3_01 = e3(0, 1), e3_11 = e3(1, 1);
      const TF e1_00 = e1(0, 0), e1_10 = e1(1, 0), e1_01 = e1(0, 1), e1_11 = e1(1, 1);
      const TF e2_00 = e2(0, 0), e2_10 = e2(1, 0), e2_01 = e2(0, 1), e2_11 = e2(1, 1);
      const double f1b2m = (double)(h * (e3_00 + e3_01)), f1b2p = (double)(h * (e3_10 + e3_11));
      const double f1b3m = (double)(-h * (e2_00 + e2_01)), f1b3p = (double)(-h * (e2_10 + e2_11));
      const double f2b1m = (double)(-h * (e3_00 + e3_10)), f2b1p = (double)(-h * (e3_01 + e3_11));
      const double f2b3m = (double)(h * (e1_00 + e1_01)), f2b3p = (double)(h * (e1_10 + e1_11));
      const double f3b1m = (double)(h * (e2_00 + e2_10)), f3b1p = (double)(h * (e2_01 + e2_11));
      const double f3b2m = (double)(-h * (e1_00 + e1_10)), f3b2p = (double)(-h * (e1_01 + e1_11));
      rhs[5] = -((f2b1p - f2b1m) * up.idx2 + (f3b1p - f3b1m) * up.idx3);
      rhs[6] = -((f1b2p - f1b2m) * up.idx1 + (f3b2p - f3b2m) * up.idx3);
      rhs[7] = -((f1b3p - f1b3m) * up.idx1 + (f2b3p - f2b3m) * up.idx2);
    }

    const int toff = tab_of(d, j, i);
    const double* ck = tab_plane(cent, d, k);
    Geo<double> g;
    if constexpr (CKS) cks_centre_geo(box, i, j, k, g);
    else load_geo(g, ck, d.ts, toff);
    if (!EARLY_PS) {
#pragma unroll
      for (int v = 0; v < NV; ++v) ps[v] = Ps[v * d.sv + c];
    }
    // geometric source S_nu = sqrt(-g) T^k_l Gamma^l_{nu k}
    {
      Fluid<double> f;
      fluid_state(ps, g, up.gam, f);
      const double eb = f.w + f.bsq, pt = f.p + 0.5 * f.bsq;
      double T[4][4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
#pragma unroll
        for (int l = 0; l < 4; ++l) T[kk][l] = eb * f.ucon[kk] * f.ucov[l] + (kk == l ? pt : 0.0) - f.bcon[kk] * f.bcov[l];
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        double sacc = 0.0;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
          for (int l = 0; l < 4; ++l) sacc += T[kk][l] * ck[(T_CONN + 10 * l + sidx(nu, kk)) * d.ts + toff];
        rhs[1 + nu] += g.gdet * sacc;
      }
    }
    double U[NV];
    {
      double pb[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) pb[v] = Pb[v * d.sv + c];
      Fluid<double> f;
      fluid_state(pb, g, up.gam, f);
      flux_of<0>(pb, f, g.gdet, U);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) U[v] = U[v] + dt * rhs[v];
    double pn[NV];
    failed = invert_1dw(U, ps, g, up.gam, pn) ? 1 : 0;
    if (up.floors) apply_floors(pn, g, ck[T_RHOFL * d.ts + toff], ck[T_UFL * d.ts + toff], up);
#pragma unroll
    for (int v = 0; v < NV; ++v) Pout[v * d.sv + c] = pn[v];
    flags[c] = (int8_t)failed;
    // Non-finite values left in the state. The hydro primitives of a zone
    // whose inversion succeeded are finite (a non-finite result is a failure,
    // and the bounds only take maxima with finite floors), and a failed zone's
    // are the fixup's to check: only the field can carry one out of here.
    if (!(isfinite(pn[5]) && isfinite(pn[6]) && isfinite(pn[7]))) atomicAdd(&ctr->bad, 1u);
  }
  block_count_to(failed, &ctr->fail, &ctr->fail_total);
}

// (256, 3): at least three waves per SIMD, i.e. at most 168 registers a lane.
// Left free the compiler takes 224 (two waves) and the kernel waits on its
// loads and long dependency chains with too little to switch to; the FP64
// variant fits 168 without spilling (the Cartesian Kerr-Schild variants,
// which evaluate the metric, spill 4 registers and still gain: their loads
// are the bound).
template <typename TF, bool DEV_DT, bool CKS = false>
__global__ __launch_bounds__(256, 3) void update_kernel(Dims d, const double* __restrict__ cent, CksBox box, UpdateParams up,
                                                     const TF* __restrict__ F1, const TF* __restrict__ F2,
                                                     const TF* __restrict__ F3, const double* Pb,
                                                     const double* __restrict__ Ps, double* Pout,
                                                     int8_t* __restrict__ flags, double dt,
                                                     const double* __restrict__ dt_dev, double dt_scale,
                                                     Counters* ctr) {
  if (DEV_DT) dt = dt_scale * *dt_dev;
  update_body<TF, false, CKS>(d, cent, box, up, F1, F2, F3, Pb, Ps, Pout, flags, dt, ctr, (int)blockIdx.x);
}

// every job of a batch: predictor P -> P_h with dt/2, corrector (P, P_h) -> P with dt
template <typename TF>
__global__ __launch_bounds__(256, 3) void update_batch_kernel(BatchView bv, int corrector) {
  const int* offs = bv.offs + PH_UPDATE * (bv.njobs + 1);
  const int jb = batch_job(offs, bv.njobs, (int)blockIdx.x);
  const JobDesc& J = bv.jobs[jb];
  const double dt = corrector ? *J.dt : 0.5 * *J.dt;
  // the FP64 batch variant runs faster with the source state loaded first (and
  // without spilling); the float-flux one and the single-job kernels slower
  update_body<TF, std::is_same<TF, double>::value>(J.d, global_ptr(J.t.cent), CksBox{}, J.up, global_ptr((const TF*)J.F[0]), global_ptr((const TF*)J.F[1]),
                  global_ptr((const TF*)J.F[2]), global_ptr(J.P), global_ptr(corrector ? J.Ph : J.P),
                  global_ptr(corrector ? J.P : J.Ph), global_ptr(J.flags), dt, global_ptr(J.ctr),
                  (int)blockIdx.x - offs[jb]);
}

// neighbour index along one direction for the fixup: across a periodic
// direction the zone on the other side of the seam, across a side whose ghost
// layer holds a neighbouring part's zones (halo bit) the ghost zone, else none
__device__ inline bool fixup_neighbour(int& x, int n, bool periodic, int halo, int lo_bit) {
  if (x >= 0 && x < n) return true;
  if (periodic) {
    x = x < 0 ? x + n : x - n;
    return true;
  }
  return (halo >> (lo_bit + (x < 0 ? 0 : 1))) & 1;
}

// failed zone <- mean of the hydro primitives of its non-failed neighbours
// among the 26 (values before any repair; across periodic directions and
// part boundaries as fixup_neighbour says), then the bounds
__device__ void fixup_body(const Dims& d, const double* __restrict__ cent, const UpdateParams& up, double* P,
                           const int8_t* __restrict__ flags, Counters* ctr, int halo, int b) {
  if (ctr->fail == 0u) return;
  const TileK tk = xcd_tile_k(b, d.utx, d.uty, d.n1, d.n3);
  const int i = tk.i0 + (int)threadIdx.x;
  const int j = tk.j0 + (int)threadIdx.y;
  const int k = tk.k;
  if (!tk.valid || i >= d.n1 || j >= d.n2) return;
  const int c = cell_of(d, k, j, i);
  if (!flags[c]) return;
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  int cnt = 0;
  for (int dk = -1; dk <= 1; ++dk)
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        if (dk == 0 && dj == 0 && di == 0) continue;
        int kk = k + dk, jj = j + dj, ii = i + di;
        if (!fixup_neighbour(ii, d.n1, up.periodic[0], halo, 0) ||
            !fixup_neighbour(jj, d.n2, up.periodic[1], halo, 2) ||
            !fixup_neighbour(kk, d.n3, up.periodic[2], halo, 4))
          continue;
        const int cc = cell_of(d, kk, jj, ii);
        if (flags[cc]) continue;
        for (int v = 0; v < 5; ++v) acc[v] += P[v * d.sv + cc];
        ++cnt;
      }
  double pn[NV];
  for (int v = 0; v < NV; ++v) pn[v] = P[v * d.sv + c];
  if (cnt > 0)
    for (int v = 0; v < 5; ++v) pn[v] = acc[v] / cnt;
  if (up.floors) {
    const int toff = tab_of(d, j, i);
    const double* ck = tab_plane(cent, d, k);
    Geo<double> g;
    load_geo(g, ck, d.ts, toff);
    apply_floors(pn, g, ck[T_RHOFL * d.ts + toff], ck[T_UFL * d.ts + toff], up);
  }
  bool fin = true;
  for (int v = 0; v < 5; ++v) {
    P[v * d.sv + c] = pn[v];
    fin = fin && isfinite(pn[v]);
  }
  if (!fin) atomicAdd(&ctr->bad, 1u);
}

// a grid of at most FIXUP_BLOCKS blocks strides over the tiles: when no zone
// failed (almost always) every block exits after one read of the counter
constexpr unsigned FIXUP_BLOCKS = 2048;  // a multiple of the XCD count
__global__ __launch_bounds__(256) void fixup_kernel(Dims d, const double* __restrict__ cent, UpdateParams up,
                                                    double* P, const int8_t* __restrict__ flags, Counters* ctr,
                                                    int halo, int ntiles) {
  if (ctr->fail == 0u) return;
  for (int b = (int)blockIdx.x; b < ntiles; b += (int)gridDim.x) fixup_body(d, cent, up, P, flags, ctr, halo, b);
}

__global__ __launch_bounds__(256) void fixup_batch_kernel(BatchView bv, int corrector) {
  const int* offs = bv.offs + PH_UPDATE * (bv.njobs + 1);
  const int jb = batch_job(offs, bv.njobs, (int)blockIdx.x);
  const JobDesc& J = bv.jobs[jb];
  fixup_body(J.d, global_ptr(J.t.cent), J.up, global_ptr(corrector ? J.P : J.Ph), global_ptr(J.flags),
             global_ptr(J.ctr), 0, (int)blockIdx.x - offs[jb]);
}

__global__ __launch_bounds__(256) void p2u_kernel(Dims d, const double* __restrict__ cent, double gam,
                                                  const double* __restrict__ P, double* __restrict__ U) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= d.n1 || j >= d.n2) return;
  const int c = cell_of(d, k, j, i);
  Geo<double> g;
  load_geo(g, tab_plane(cent, d, k), d.ts, tab_of(d, j, i));
  double p[NV], u[NV];
  for (int v = 0; v < NV; ++v) p[v] = P[v * d.sv + c];
  Fluid<double> f;
  fluid_state(p, g, gam, f);
  flux_of<0>(p, f, g.gdet, u);
  for (int v = 0; v < NV; ++v) U[v * d.sv + c] = u[v];
}

__global__ __launch_bounds__(256) void u2p_kernel(Dims d, const double* __restrict__ cent, UpdateParams up,
                                                  const double* __restrict__ U, double* __restrict__ P,
                                                  int8_t* __restrict__ flags, Counters* ctr) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j = blockIdx.y * 4 + threadIdx.y;
  const int k = blockIdx.z;
  int failed = 0;
  if (i < d.n1 && j < d.n2) {
    const int c = cell_of(d, k, j, i);
    const int toff = tab_of(d, j, i);
    const double* ck = tab_plane(cent, d, k);
    Geo<double> g;
    load_geo(g, ck, d.ts, toff);
    double u[NV], guess[NV], pn[NV];
    for (int v = 0; v < NV; ++v) {
      u[v] = U[v * d.sv + c];
      guess[v] = P[v * d.sv + c];
    }
    failed = invert_1dw(u, guess, g, up.gam, pn) ? 1 : 0;
    if (up.floors) apply_floors(pn, g, ck[T_RHOFL * d.ts + toff], ck[T_UFL * d.ts + toff], up);
    for (int v = 0; v < NV; ++v) P[v * d.sv + c] = pn[v];
    flags[c] = (int8_t)failed;
  }
  block_count_to(failed, &ctr->fail);
}

}  // namespace

hipError_t launch_update(bool mixed, const Dims& d, const Tables& t, const UpdateParams& up, const void* F1,
                         const void* F2, const void* F3, const double* Pb, const double* Ps, double* Pout,
                         int8_t* flags, double dt, const double* dt_dev, double dt_scale, Counters* ctr,
                         hipStream_t s, const grmhd_problem* cks) {
  const unsigned nblk = xcd_grid(d.n1, d.n2, d.n3, d.utx, d.uty);
  dim3 blk(d.utx, d.uty, 1), grd(nblk);
  const CksBox box = cks ? cks_box(*cks) : CksBox{};
  if (mixed) {
    const float *f1 = (const float*)F1, *f2 = (const float*)F2, *f3 = (const float*)F3;
    if (cks && dt_dev)
      hipLaunchKernelGGL((update_kernel<float, true, true>), grd, blk, 0, s, d, t.cent, box, up, f1, f2, f3, Pb, Ps,
                         Pout, flags, dt, dt_dev, dt_scale, ctr);
    else if (cks)
      hipLaunchKernelGGL((update_kernel<float, false, true>), grd, blk, 0, s, d, t.cent, box, up, f1, f2, f3, Pb, Ps,
                         Pout, flags, dt, dt_dev, dt_scale, ctr);
    else if (dt_dev)
      hipLaunchKernelGGL((update_kernel<float, true>), grd, blk, 0, s, d, t.cent, box, up, f1, f2, f3, Pb, Ps, Pout,
                         flags, dt, dt_dev, dt_scale, ctr);
    else
      hipLaunchKernelGGL((update_kernel<float, false>), grd, blk, 0, s, d, t.cent, box, up, f1, f2, f3, Pb, Ps, Pout,
                         flags, dt, dt_dev, dt_scale, ctr);
  } else {
    const double *f1 = (const double*)F1, *f2 = (const double*)F2, *f3 = (const double*)F3;
    if (cks && dt_dev)
      hipLaunchKernelGGL((update_kernel<double, true, true>), grd, blk, 0, s, d, t.cent, box, up, f1, f2, f3, Pb, Ps,
                         Pout, flags, dt, dt_dev, dt_scale, ctr);
    else if (cks)
      hipLaunchKernelGGL((update_kernel<double, false, true>), grd, blk, 0, s, d, t.cent, box, up, f1, f2, f3, Pb, Ps,
                         Pout, flags, dt, dt_dev, dt_scale, ctr);
    else if (dt_dev)
      hipLaunchKernelGGL((update_kernel<double, true>), grd, blk, 0, s, d, t.cent, box, up, f1, f2, f3, Pb, Ps, Pout,
                         flags, dt, dt_dev, dt_scale, ctr);
    else
      hipLaunchKernelGGL((update_kernel<double, false>), grd, blk, 0, s, d, t.cent, box, up, f1, f2, f3, Pb, Ps, Pout,
                         flags, dt, dt_dev, dt_scale, ctr);
  }
  return hipGetLastError();
}

hipError_t launch_fixup(const Dims& d, const Tables& t, const UpdateParams& up, double* P, const int8_t* flags,
                        Counters* ctr, int halo, hipStream_t s) {
  const unsigned ntiles = xcd_grid(d.n1, d.n2, d.n3, d.utx, d.uty);
  const unsigned nblk = ntiles < FIXUP_BLOCKS ? ntiles : FIXUP_BLOCKS;
  hipLaunchKernelGGL(fixup_kernel, dim3(nblk), dim3(d.utx, d.uty, 1), 0, s, d, t.cent, up, P, flags, ctr, halo,
                     (int)ntiles);
  return hipGetLastError();
}

hipError_t launch_batch_update(const BatchView& bv, const int* totals, bool mixed, bool corrector, int which,
                               hipStream_t s) {
  const dim3 blk(bv.utx, bv.uty, 1), grd(totals[PH_UPDATE]);
  const int c = corrector ? 1 : 0;
  if (which & 1) {
    if (mixed) hipLaunchKernelGGL(update_batch_kernel<float>, grd, blk, 0, s, bv, c);
    else hipLaunchKernelGGL(update_batch_kernel<double>, grd, blk, 0, s, bv, c);
  }
  if (which & 2) hipLaunchKernelGGL(fixup_batch_kernel, grd, blk, 0, s, bv, c);
  return hipGetLastError();
}

hipError_t launch_prim_to_cons(const Dims& d, const Tables& t, double gam, const double* P, double* U,
                               hipStream_t s) {
  dim3 blk(64, 4, 1), grd((d.n1 + 63) / 64, (d.n2 + 3) / 4, d.n3);
  hipLaunchKernelGGL(p2u_kernel, grd, blk, 0, s, d, t.cent, gam, P, U);
  return hipGetLastError();
}

hipError_t launch_cons_to_prim(const Dims& d, const Tables& t, const UpdateParams& up, const double* U,
                               double* P, int8_t* flags, Counters* ctr, hipStream_t s) {
  dim3 blk(64, 4, 1), grd((d.n1 + 63) / 64, (d.n2 + 3) / 4, d.n3);
  hipLaunchKernelGGL(u2p_kernel, grd, blk, 0, s, d, t.cent, up, U, P, flags, ctr);
  return hipGetLastError();
}
