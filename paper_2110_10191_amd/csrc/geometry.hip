// Geometry tables: metric, inverse, sqrt(-g) and lapse at zone centres and
// faces; connection at centres by centred differences of the metric; floor
// scales. Implementation Notes section: every metric-dependent quantity is
// evaluated numerically from an analytic line element, the coordinates act as
// static mesh refinement (MKS / funky MKS concentrate zones towards the disk
// midplane), and another coordinate system or stationary spacetime is a small
// change: Cartesian Kerr-Schild (metric eta + f l l in (t, x, y, z)) makes
// every table depend on x3, so its tables are 3D with an x3-face table.
#include "kernels.h"
#include "cks_geometry.h"

// No fused multiply-adds here: the connection's centred differences (step
// 1e-5) turn a one-ulp change of the metric into a 1e-10 change of Gamma, so
// every table value is the plain sequence of correctly rounded operations its
// formula spells out.
#pragma clang fp contract(off)

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

// Cartesian Kerr-Schild: g = eta + f l l with f = 2 r^3 / (r^4 + a^2 z^2) and
// the null covector l = (1, (r x + a y)/(r^2 + a^2), (r y - a x)/(r^2 + a^2), z/r)
__device__ void gcov_cks(double x, double y, double z, double a, double g[4][4]) {
  const double r = cks_radius(x, y, z, a);
  const double r2 = r * r;
  const double f = 2.0 * r2 * r / (r2 * r2 + a * a * z * z);
  const double ra = r2 + a * a;
  const double l[4] = {1.0, (r * x + a * y) / ra, (r * y - a * x) / ra, z / r};
  for (int m = 0; m < 4; ++m)
    for (int n = 0; n < 4; ++n) g[m][n] = f * l[m] * l[n] + (m != n ? 0.0 : (m == 0 ? -1.0 : 1.0));
}

// covariant metric in code coordinates, full 4x4
__device__ void gcov_code(double x1, double x2, double x3, const grmhd_problem& p, double g[4][4]) {
  if (p.coords == GRMHD_KERR_CKS) {
    gcov_cks(x1, x2, x3, p.a, g);
    return;
  }
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

// write metric, inverse (upper triangle), sqrt(-g) and lapse of one point:
// into the centre table (dt, one plane per component; ft null) or into a face
// table and its float copy (paired components)
__device__ void store_point(double x1, double x2, double x3, const grmhd_problem& p, double* dt, float* ft,
                            size_t ts, int off, double gcon_out[4][4]) {
  double g[4][4], gi[4][4];
  gcov_code(x1, x2, x3, p, g);
  const double det = invert4(g, gi);
  auto at = [&](int c) -> size_t { return ft ? pair_index(c, ts, (size_t)off) : (size_t)c * ts + (size_t)off; };
  for (int m = 0; m < 4; ++m)
    for (int n = m; n < 4; ++n) {
      const int c = sidx(m, n);
      dt[at(T_GCOV + c)] = g[m][n];
      dt[at(T_GCON + c)] = gi[m][n];
      if (ft) {
        ft[at(T_GCOV + c)] = (float)g[m][n];
        ft[at(T_GCON + c)] = (float)gi[m][n];
      }
    }
  const double gdet = sqrt(fabs(det));
  const double alpha = 1.0 / sqrt(-gi[0][0]);
  dt[at(T_GDET)] = gdet;
  dt[at(T_ALPHA)] = alpha;
  if (ft) {
    ft[at(T_GDET)] = (float)gdet;
    ft[at(T_ALPHA)] = (float)alpha;
  }
  if (gcon_out)
    for (int m = 0; m < 4; ++m)
      for (int n = 0; n < 4; ++n) gcon_out[m][n] = gi[m][n];
}

// a face table entry (paired components) and its float copy
__device__ void store_face(const Geo<double>& g, double* dt, float* ft, size_t ts, int off) {
  for (int c = 0; c < 10; ++c) {
    dt[pair_index(T_GCOV + c, ts, (size_t)off)] = g.gcov[c];
    dt[pair_index(T_GCON + c, ts, (size_t)off)] = g.gcon[c];
    ft[pair_index(T_GCOV + c, ts, (size_t)off)] = (float)g.gcov[c];
    ft[pair_index(T_GCON + c, ts, (size_t)off)] = (float)g.gcon[c];
  }
  dt[pair_index(T_GDET, ts, (size_t)off)] = g.gdet;
  dt[pair_index(T_ALPHA, ts, (size_t)off)] = g.alpha;
  ft[pair_index(T_GDET, ts, (size_t)off)] = (float)g.gdet;
  ft[pair_index(T_ALPHA, ts, (size_t)off)] = (float)g.alpha;
}

__global__ void geometry_kernel(grmhd_problem p, Dims d, Tables t, CksBox box) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x) - NG;
  const int j = (int)(blockIdx.y * blockDim.y + threadIdx.y) - NG;
  const int k = (int)blockIdx.z - NG;  // 2D tables: a single plane (k = -NG, tk = 0)
  if (i >= d.n1 + NG || j >= d.n2 + NG) return;
  const int off = (k + NG) * d.tk + tab_of(d, j, i);
  const size_t ts = (size_t)d.ts;
  const double dx1 = (p.x1max - p.x1min) / p.n1;
  const double dx2 = (p.x2max - p.x2min) / p.n2;
  const double dx3 = (p.x3max - p.x3min) / p.n3;
  const double x1c = p.x1min + (i + 0.5) * dx1, x2c = p.x2min + (j + 0.5) * dx2, x3c = p.x3min + (k + 0.5) * dx3;
  const double x1f = p.x1min + i * dx1, x2f = p.x2min + j * dx2;
  const bool k3 = p.coords == GRMHD_KERR_CKS;

  double gcon[4][4];
  if (k3) {
    // Cartesian Kerr-Schild centres in closed form, the values the update
    // computes itself (the connection below uses this inverse)
    Geo<double> g;
    cks_centre_geo(box, i, j, k, g);
    for (int c = 0; c < 10; ++c) {
      t.cent[(size_t)(T_GCOV + c) * ts + off] = g.gcov[c];
      t.cent[(size_t)(T_GCON + c) * ts + off] = g.gcon[c];
    }
    t.cent[(size_t)T_GDET * ts + off] = g.gdet;
    t.cent[(size_t)T_ALPHA * ts + off] = g.alpha;
    for (int m = 0; m < 4; ++m)
      for (int n = 0; n < 4; ++n) gcon[m][n] = g.gcon[sidx(m, n)];
  } else {
    store_point(x1c, x2c, x3c, p, t.cent, nullptr, ts, off, gcon);
  }
  if (k3) {
    // Cartesian Kerr-Schild faces in closed form, the values the face-flux
    // pass computes itself
    // box: the zone corner and widths the face-flux pass uses (computed on the host)
    const CksBox& b = box;
    double* const dt[3] = {t.f1, t.f2, t.f3};
    float* const ft[3] = {t.f1f, t.f2f, t.f3f};
    for (int D = 1; D <= 3; ++D) {
      Geo<double> g;
      cks_face_geo(b, D, i, j, k, g);
      store_face(g, dt[D - 1], ft[D - 1], ts, off);
    }
  } else {
    store_point(x1f, x2c, x3c, p, t.f1, t.f1f, ts, off, nullptr);
    store_point(x1c, x2f, x3c, p, t.f2, t.f2f, ts, off, nullptr);
    // 2D tables: the metric does not depend on x3, and the x3-face table
    // holds the centre values
    store_point(x1c, x2c, x3c, p, t.f3, t.f3f, ts, off, nullptr);
  }

  // connection: Gamma_kmn = (d_n g_km + d_m g_kn - d_k g_mn)/2, Gamma^l_mn = g^lk Gamma_kmn,
  // derivatives by centred differences in x1, x2 and (3D tables) x3; d_t = 0
  double dg[3][4][4];  // dg[c-1][a][b] = d_c g_ab, c = 1..3
  for (int c = 0; c < 3; ++c)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) dg[c][a][b] = 0.0;
  if (p.coords != GRMHD_MINKOWSKI_CART) {
    const int nd = k3 ? 3 : 2;
    for (int c = 0; c < nd; ++c) {
      const double e1 = c == 0 ? FD_DELTA : 0.0, e2 = c == 1 ? FD_DELTA : 0.0, e3 = c == 2 ? FD_DELTA : 0.0;
      double gp[4][4], gm[4][4];
      gcov_code(x1c + e1, x2c + e2, x3c + e3, p, gp);
      gcov_code(x1c - e1, x2c - e2, x3c - e3, p, gm);
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) dg[c][a][b] = (gp[a][b] - gm[a][b]) / (2.0 * FD_DELTA);
    }
  }
  auto D = [&](int c, int a, int b) -> double { return c > 0 ? dg[c - 1][a][b] : 0.0; };
  for (int l = 0; l < 4; ++l)
    for (int m = 0; m < 4; ++m)
      for (int n = m; n < 4; ++n) {
        double s = 0.0;
        for (int q = 0; q < 4; ++q) s += gcon[l][q] * 0.5 * (D(n, q, m) + D(m, q, n) - D(q, m, n));
        t.cent[(T_CONN + 10 * l + sidx(m, n)) * ts + off] = s;
      }

  // floor scales: k = 1/(r^2 (1 + r/10)) with r = exp(x1) (MKS / FMKS) or the
  // Kerr-Schild radius of the Cartesian point
  double rfl = 0.0, ufl = 0.0;
  if (p.coords != GRMHD_MINKOWSKI_CART) {
    const double r = k3 ? cks_radius(x1c, x2c, x3c, p.a) : exp(x1c);
    const double kk = 1.0 / (r * r * (1.0 + r / 10.0));
    rfl = p.rho_fl * kk;
    ufl = p.u_fl * pow(kk, p.gam);
  }
  t.cent[T_RHOFL * ts + off] = rfl;
  t.cent[T_UFL * ts + off] = ufl;
}

}  // namespace

hipError_t launch_geometry(const grmhd_problem& p, const Dims& d, const Tables& t, hipStream_t s) {
  dim3 blk(64, 4, 1);
  dim3 grd((d.n1 + 2 * NG + 63) / 64, (d.n2 + 2 * NG + 3) / 4, d.tk ? d.p3 : 1);
  hipLaunchKernelGGL(geometry_kernel, grd, blk, 0, s, p, d, t, cks_box(p));
  return hipGetLastError();
}
