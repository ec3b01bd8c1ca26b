// Cartesian Kerr-Schild geometry of a point in closed form, for the face
// tables and the metric part of the centre table, and for the face-flux pass
// and the update, which compute it instead of reading it. Implementation Notes section: a change of coordinates or background
// spacetime only changes the metric evaluation. The metric is
// g = eta + f l l with f = 2 r^3 / (r^4 + a^2 z^2) and the covector
// l = (1, (r x + a y)/(r^2 + a^2), (r y - a x)/(r^2 + a^2), z/r), null for
// both eta and g; hence g^-1 = eta - f l^ l^ with l^ = (-1, l1, l2, l3),
// det g = -1 (sqrt(-g) = 1) and the lapse 1/sqrt(-g^tt) = 1/sqrt(1 + f).
// Both users evaluate the same operations without contraction, so the values
// are the same bits wherever they come from.
#pragma once

#include "common.h"

struct CksBox {
  double x0[3];  // x1min, x2min, x3min
  double dx[3];  // zone widths
  double a;
};

// on the host, so that every user of the box has the same bits
inline CksBox cks_box(const grmhd_problem& p) {
  CksBox b;
  b.x0[0] = p.x1min;
  b.x0[1] = p.x2min;
  b.x0[2] = p.x3min;
  b.dx[0] = (p.x1max - p.x1min) / p.n1;
  b.dx[1] = (p.x2max - p.x2min) / p.n2;
  b.dx[2] = (p.x3max - p.x3min) / p.n3;
  b.a = p.a;
  return b;
}

// the positive root r of r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0, R^2 = x^2 + y^2 + z^2
__device__ inline double cks_radius(double x, double y, double z, double a) {
#pragma clang fp contract(off)
  const double h = 0.5 * (x * x + y * y + z * z - a * a);
  return sqrt(h + sqrt(h * h + a * a * z * z));
}

// metric, inverse, sqrt(-g) and lapse at the point (x, y, z); double
// precision, stored as T
template <typename T>
__device__ inline void cks_point_geo(double x, double y, double z, double a, Geo<T>& g) {
#pragma clang fp contract(off)
  const double r = cks_radius(x, y, z, a);
  const double r2 = r * r;
  const double f = 2.0 * r2 * r / (r2 * r2 + a * a * z * z);
  const double ra = r2 + a * a;
  const double l[4] = {1.0, (r * x + a * y) / ra, (r * y - a * x) / ra, z / r};
  const double lu[4] = {-1.0, l[1], l[2], l[3]};
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int n = m; n < 4; ++n) {
      const double eta = m != n ? 0.0 : (m == 0 ? -1.0 : 1.0);
      g.gcov[sidx(m, n)] = (T)(f * l[m] * l[n] + eta);
      g.gcon[sidx(m, n)] = (T)(eta - f * lu[m] * lu[n]);
    }
  // sqrt(-g) = 1, held in a register the compiler cannot see through: a
  // known 1 would let it drop the products with sqrt(-g) and fuse the
  // remaining operations differently from the same code reading the value
  // from a table, and the two must round alike
  double one = 1.0;
  asm volatile("" : "+v"(one));
  g.gdet = (T)one;
  g.alpha = (T)(1.0 / sqrt(1.0 + f));
}

// at the lower D-face (D = 1..3) of cell (i, j, k)
template <typename T>
__device__ inline void cks_face_geo(const CksBox& b, int D, int i, int j, int k, Geo<T>& g) {
#pragma clang fp contract(off)
  const double x = b.x0[0] + (D == 1 ? (double)i : i + 0.5) * b.dx[0];
  const double y = b.x0[1] + (D == 2 ? (double)j : j + 0.5) * b.dx[1];
  const double z = b.x0[2] + (D == 3 ? (double)k : k + 0.5) * b.dx[2];
  cks_point_geo(x, y, z, b.a, g);
}

// at the centre of cell (i, j, k)
template <typename T>
__device__ inline void cks_centre_geo(const CksBox& b, int i, int j, int k, Geo<T>& g) {
#pragma clang fp contract(off)
  const double x = b.x0[0] + (i + 0.5) * b.dx[0];
  const double y = b.x0[1] + (j + 0.5) * b.dx[1];
  const double z = b.x0[2] + (k + 0.5) * b.dx[2];
  cks_point_geo(x, y, z, b.a, g);
}
