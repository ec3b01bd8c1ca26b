// Geometry tables: metric, inverse, sqrt(-g) and lapse at zone centres and x1/x2
// faces; connection at centres by centred differences of the metric; floor
// scales. Implementation Notes section: every metric-dependent quantity is
// evaluated numerically from an analytic line element, and the coordinates act
// as static mesh refinement (MKS / funky MKS concentrate zones towards the
// disk midplane).
#include "kernels.h"

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr double FD_DELTA = 1e-5;
constexpr double SIN_MIN = 1e-20;  // |sin theta| floor inside the metric (polar faces)

// theta(x1, x2) of MKS / funky MKS
__device__ double theta_of(double x1, double x2, const grmhd_problem& p) {
  const double tg = PI * x2 + 0.5 * (1.0 - p.hslope) * sin(2.0 * PI * x2);
  if (p.coords == GRMHD_KERR_MKS) return tg;
  const double al = p.poly_alpha, xt = p.poly_xt;
  const double norm = 0.5 * PI / (1.0 + 1.0 / ((al + 1.0) * pow(xt, al)));
  const double y = 2.0 * x2 - 1.0;
  const double tj = norm * y * (1.0 + pow(y / xt, al) / (al + 1.0)) + 0.5 * PI;
  return tg + exp(-p.mks_smooth * (x1 - p.x1min)) * (tj - tg);
}

__device__ void theta_derivs(double x1, double x2, const grmhd_problem& p, double& d1, double& d2) {
  const double dtg = PI * (1.0 + (1.0 - p.hslope) * cos(2.0 * PI * x2));
  if (p.coords == GRMHD_KERR_MKS) {
    d1 = 0.0;
    d2 = dtg;
    return;
  }
  const double tg = PI * x2 + 0.5 * (1.0 - p.hslope) * sin(2.0 * PI * x2);
  const double al = p.poly_alpha, xt = p.poly_xt;
  const double norm = 0.5 * PI / (1.0 + 1.0 / ((al + 1.0) * pow(xt, al)));
  const double y = 2.0 * x2 - 1.0;
  const double yp = pow(y / xt, al);
  const double tj = norm * y * (1.0 + yp / (al + 1.0)) + 0.5 * PI;
  const double dtj = 2.0 * norm * (1.0 + yp);
  const double e = exp(-p.mks_smooth * (x1 - p.x1min));
  d1 = -p.mks_smooth * e * (tj - tg);
  d2 = dtg + e * (dtj - dtg);
}

// covariant metric in code coordinates, full 4x4
__device__ void gcov_code(double x1, double x2, const grmhd_problem& p, double g[4][4]) {
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) g[m][n] = 0.0;
  if (p.coords == GRMHD_MINKOWSKI_CART) {
    g[0][0] = -1.0;
    g[1][1] = g[2][2] = g[3][3] = 1.0;
    return;
  }
  const double a = p.a;
  const double r = exp(x1);
  const double th = theta_of(x1, x2, p);
  double d1, d2;
  theta_derivs(x1, x2, p, d1, d2);
  double sth = sin(th);
  if (fabs(sth) < SIN_MIN) sth = SIN_MIN;
  const double s2 = sth * sth;
  const double cth = cos(th);
  const double rho2 = r * r + a * a * cth * cth;
  const double f = 2.0 * r / rho2;
  // Kerr-Schild (t, r, theta, phi)
  const double ktt = -(1.0 - f), ktr = f, ktp = -a * f * s2, krr = 1.0 + f;
  const double krp = -a * s2 * (1.0 + f), khh = rho2, kpp = s2 * (rho2 + a * a * s2 * (1.0 + f));
  // J: r = exp(x1) -> dr/dx1 = r; theta(x1, x2); phi = x3
  g[0][0] = ktt;
  g[0][1] = g[1][0] = ktr * r;
  g[0][3] = g[3][0] = ktp;
  g[1][1] = krr * r * r + khh * d1 * d1;
  g[1][2] = g[2][1] = khh * d1 * d2;
  g[1][3] = g[3][1] = krp * r;
  g[2][2] = khh * d2 * d2;
  g[3][3] = kpp;
}

// inverse and determinant by expansion in complementary 2x2 minors
__device__ double invert4(const double m[4][4], double b[4][4]) {
  const double s0 = m[0][0] * m[1][1] - m[1][0] * m[0][1];
  const double s1 = m[0][0] * m[1][2] - m[1][0] * m[0][2];
  const double s2 = m[0][0] * m[1][3] - m[1][0] * m[0][3];
  const double s3 = m[0][1] * m[1][2] - m[1][1] * m[0][2];
  const double s4 = m[0][1] * m[1][3] - m[1][1] * m[0][3];
  const double s5 = m[0][2] * m[1][3] - m[1][2] * m[0][3];
  const double c5 = m[2][2] * m[3][3] - m[3][2] * m[2][3];
  const double c4 = m[2][1] * m[3][3] - m[3][1] * m[2][3];
  const double c3 = m[2][1] * m[3][2] - m[3][1] * m[2][2];
  const double c2 = m[2][0] * m[3][3] - m[3][0] * m[2][3];
  const double c1 = m[2][0] * m[3][2] - m[3][0] * m[2][2];
  const double c0 = m[2][0] * m[3][1] - m[3][0] * m[2][1];
  const double det = s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0;
  const double id = 1.0 / det;
  b[0][0] = (m[1][1] * c5 - m[1][2] * c4 + m[1][3] * c3) * id;
  b[0][1] = (-m[0][1] * c5 + m[0][2] * c4 - m[0][3] * c3) * id;
  b[0][2] = (m[3][1] * s5 - m[3][2] * s4 + m[3][3] * s3) * id;
  b[0][3] = (-m[2][1] * s5 + m[2][2] * s4 - m[2][3] * s3) * id;
  b[1][0] = (-m[1][0] * c5 + m[1][2] * c2 - m[1][3] * c1) * id;
  b[1][1] = (m[0][0] * c5 - m[0][2] * c2 + m[0][3] * c1) * id;
  b[1][2] = (-m[3][0] * s5 + m[3][2] * s2 - m[3][3] * s1) * id;
  b[1][3] = (m[2][0] * s5 - m[2][2] * s2 + m[2][3] * s1) * id;
  b[2][0] = (m[1][0] * c4 - m[1][1] * c2 + m[1][3] * c0) * id;
  b[2][1] = (-m[0][0] * c4 + m[0][1] * c2 - m[0][3] * c0) * id;
  b[2][2] = (m[3][0] * s4 - m[3][1] * s2 + m[3][3] * s0) * id;
  b[2][3] = (-m[2][0] * s4 + m[2][1] * s2 - m[2][3] * s0) * id;
  b[3][0] = (-m[1][0] * c3 + m[1][1] * c1 - m[1][2] * c0) * id;
  b[3][1] = (m[0][0] * c3 - m[0][1] * c1 + m[0][2] * c0) * id;
  b[3][2] = (-m[3][0] * s3 + m[3][1] * s1 - m[3][2] * s0) * id;
  b[3][3] = (m[2][0] * s3 - m[2][1] * s1 + m[2][2] * s0) * id;
  return det;
}

// write metric, inverse (upper triangle), sqrt(-g) and lapse of one point
__device__ void store_point(double x1, double x2, const grmhd_problem& p, double* dt, float* ft,
                            int ts, int off, double gcon_out[4][4]) {
  double g[4][4], gi[4][4];
  gcov_code(x1, x2, p, g);
  const double det = invert4(g, gi);
  for (int m = 0; m < 4; ++m)
    for (int n = m; n < 4; ++n) {
      const int c = sidx(m, n);
      dt[(T_GCOV + c) * ts + off] = g[m][n];
      dt[(T_GCON + c) * ts + off] = gi[m][n];
      ft[(T_GCOV + c) * ts + off] = (float)g[m][n];
      ft[(T_GCON + c) * ts + off] = (float)gi[m][n];
    }
  const double gdet = sqrt(fabs(det));
  const double alpha = 1.0 / sqrt(-gi[0][0]);
  dt[T_GDET * ts + off] = gdet;
  dt[T_ALPHA * ts + off] = alpha;
  ft[T_GDET * ts + off] = (float)gdet;
  ft[T_ALPHA * ts + off] = (float)alpha;
  if (gcon_out)
    for (int m = 0; m < 4; ++m)
      for (int n = 0; n < 4; ++n) gcon_out[m][n] = gi[m][n];
}

__global__ void geometry_kernel(grmhd_problem p, Dims d, Tables t) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x) - NG;
  const int j = (int)(blockIdx.y * blockDim.y + threadIdx.y) - NG;
  if (i >= d.n1 + NG || j >= d.n2 + NG) return;
  const int off = tab_of(d, j, i);
  const double dx1 = (p.x1max - p.x1min) / p.n1;
  const double dx2 = (p.x2max - p.x2min) / p.n2;
  const double x1c = p.x1min + (i + 0.5) * dx1, x2c = p.x2min + (j + 0.5) * dx2;
  const double x1f = p.x1min + i * dx1, x2f = p.x2min + j * dx2;

  double gcon[4][4];
  store_point(x1c, x2c, p, t.cent, t.centf, d.ts, off, gcon);
  store_point(x1f, x2c, p, t.f1, t.f1f, d.ts, off, nullptr);
  store_point(x1c, x2f, p, t.f2, t.f2f, d.ts, off, nullptr);

  // connection: Gamma_kmn = (d_n g_km + d_m g_kn - d_k g_mn)/2, Gamma^l_mn = g^lk Gamma_kmn,
  // derivatives by centred differences in x1 and x2 (d_t = d_x3 = 0)
  double dg[3][4][4];  // dg[c-1][a][b] = d_c g_ab for c = 1, 2; index 2 unused (zero)
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) dg[2][a][b] = 0.0;
  if (p.coords != GRMHD_MINKOWSKI_CART) {
    double gp[4][4], gm[4][4];
    gcov_code(x1c + FD_DELTA, x2c, p, gp);
    gcov_code(x1c - FD_DELTA, x2c, p, gm);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) dg[0][a][b] = (gp[a][b] - gm[a][b]) / (2.0 * FD_DELTA);
    gcov_code(x1c, x2c + FD_DELTA, p, gp);
    gcov_code(x1c, x2c - FD_DELTA, p, gm);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) dg[1][a][b] = (gp[a][b] - gm[a][b]) / (2.0 * FD_DELTA);
  } else {
    for (int c = 0; c < 2; ++c)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) dg[c][a][b] = 0.0;
  }
  auto D = [&](int c, int a, int b) -> double { return (c == 1 || c == 2) ? dg[c - 1][a][b] : 0.0; };
  for (int l = 0; l < 4; ++l)
    for (int m = 0; m < 4; ++m)
      for (int n = m; n < 4; ++n) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) s += gcon[l][k] * 0.5 * (D(n, k, m) + D(m, k, n) - D(k, m, n));
        t.cent[(T_CONN + 10 * l + sidx(m, n)) * d.ts + off] = s;
      }

  // floor scales (Kerr: r = exp(x1))
  double rfl = 0.0, ufl = 0.0;
  if (p.coords != GRMHD_MINKOWSKI_CART) {
    const double r = exp(x1c);
    const double k = 1.0 / (r * r * (1.0 + r / 10.0));
    rfl = p.rho_fl * k;
    ufl = p.u_fl * pow(k, p.gam);
  }
  t.cent[T_RHOFL * d.ts + off] = rfl;
  t.cent[T_UFL * d.ts + off] = ufl;
}

}  // namespace

hipError_t launch_geometry(const grmhd_problem& p, const Dims& d, const Tables& t, hipStream_t s) {
  dim3 blk(64, 4, 1);
  dim3 grd((d.n1 + 2 * NG + 63) / 64, (d.n2 + 2 * NG + 3) / 4, 1);
  hipLaunchKernelGGL(geometry_kernel, grd, blk, 0, s, p, d, t);
  return hipGetLastError();
}
