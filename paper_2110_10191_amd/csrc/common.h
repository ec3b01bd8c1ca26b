// Shared device definitions of the GRMHD zone-update library (gfx950).
//
// Layout (see grmhd.h): a state is [8][n3+6][n2+6][n1p] float64, x1 fastest.
// Face fluxes use the same layout: F_d at cell (k, j, i) is the flux through
// the lower d-face of that cell. Geometry tables hold centre quantities
// (metric, inverse, sqrt(-g), lapse, connection, floor scales) and face
// quantities (metric, inverse, sqrt(-g), lapse) per direction. Axisymmetric
// coordinates store them as 2D tables [component][n2+6][n1p] (k stride 0),
// and the x3 faces share the centre geometry; Cartesian Kerr-Schild, whose
// metric depends on x3, stores 3D tables [component][n3+6][n2+6][n1p] (k
// stride = the state's) with an x3-face table of its own.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "grmhd.h"

#define NG GRMHD_NG
#define NV GRMHD_NVAR

// geometry table components
enum {
  T_GCOV = 0,     // 10: symmetric g_mn, order 00 01 02 03 11 12 13 22 23 33
  T_GCON = 10,    // 10: g^mn, same order
  T_GDET = 20,
  T_ALPHA = 21,
  N_FACE = 22,
  T_CONN = 22,    // 40: Gamma^l_mn, l-major, (m,n) in the symmetric order
  T_RHOFL = 62,   // rho_fl * k        (k = 1/(r^2 (1 + r/10)))
  T_UFL = 63,     // u_fl * k^gamma
  N_CENT = 64
};

__host__ __device__ constexpr int sidx(int m, int n) {
  return (m <= n) ? (m * 4 - (m * (m - 1)) / 2 + (n - m)) : (n * 4 - (n * (n - 1)) / 2 + (m - n));
}

struct Dims {
  int n1, n2, n3;
  int p1, p2, p3;  // padded extents: n1p, n2 + 6, n3 + 6
  int s2;          // j stride (= p1)
  int s3;          // k stride (= p2 * p1)
  int sv;          // variable stride (= p3 * p2 * p1)
  int ts;          // table component stride (p2 * p1, or p3 * p2 * p1 for 3D tables)
  int tk;          // table k stride (0 for 2D tables, s3 for 3D)
  int stx, sty;    // thread-block tile (x1 x x2) of the sweeps
  int utx, uty;    // thread-block tile of the update and fixup
  int out_lo, out_hi;  // x1 lower / upper boundary is an outflow boundary
};

__host__ __device__ inline int cell_of(const Dims& d, int k, int j, int i) {
  return (k + NG) * d.s3 + (j + NG) * d.s2 + (i + NG);
}
// point index of (j, i) within one x3 plane of the tables; tab_plane gives the
// plane of x3 index k (the only plane of 2D tables)
__host__ __device__ inline int tab_of(const Dims& d, int j, int i) { return (j + NG) * d.s2 + (i + NG); }
template <typename S>
__host__ __device__ inline const S* tab_plane(const S* tab, const Dims& d, int k) {
  return tab + (size_t)(k + NG) * (size_t)d.tk;
}

// Loads as (wave-uniform base pointer) + (32-bit unsigned byte offset):
// the backend can then keep the base in scalar registers and share one 32-bit
// vector offset across all components, instead of a 64-bit vector address per
// load. Every array here is < 4 GiB per component (checked at init).
template <typename S>
__device__ inline S ldu(const S* base, unsigned byte_off) {
  return *(const S*)((const char*)base + byte_off);
}
// The face tables hold their components in pairs: component c of point off
// at (c & ~1) * ts + 2 * off + (c & 1), so one 16-byte (FP64) or 8-byte
// (FP32) load per lane brings two components. The centre table keeps one
// plane per component (c * ts + off).
__host__ __device__ inline size_t pair_index(int c, size_t ts, size_t off) {
  return (size_t)(c & ~1) * ts + 2 * off + (size_t)(c & 1);
}
template <typename S>
__host__ __device__ inline const S* face_plane(const S* tab, const Dims& d, int k) {
  return tab + 2 * (size_t)(k + NG) * (size_t)d.tk;
}
template <typename S>
struct pair_of;
template <>
struct pair_of<double> {
  using type = double2;
};
template <>
struct pair_of<float> {
  using type = float2;
};

template <typename T>
struct Geo {
  T gcov[10];
  T gcon[10];
  T gdet;
  T alpha;
};

// centre table: component c lives at tab + c * ts; off is the point index (tab_of)
template <typename T, typename S>
__device__ inline void load_geo(Geo<T>& g, const S* __restrict__ tab, int ts, int off) {
  const unsigned bo = (unsigned)off * (unsigned)sizeof(S);
#pragma unroll
  for (int c = 0; c < 10; ++c) g.gcov[c] = (T)ldu(tab + (size_t)(T_GCOV + c) * ts, bo);
#pragma unroll
  for (int c = 0; c < 10; ++c) g.gcon[c] = (T)ldu(tab + (size_t)(T_GCON + c) * ts, bo);
  g.gdet = (T)ldu(tab + (size_t)T_GDET * ts, bo);
  g.alpha = (T)ldu(tab + (size_t)T_ALPHA * ts, bo);
}

// the same from a face table (paired components; off as above, tab the plane
// from face_plane)
template <typename T, typename S>
__device__ inline void load_face_geo(Geo<T>& g, const S* __restrict__ tab, int ts, int off) {
  using P2 = typename pair_of<S>::type;
  const unsigned bo = (unsigned)off * (unsigned)(2 * sizeof(S));
  auto ld = [&](int c0) -> P2 { return *(const P2*)((const char*)(tab + (size_t)c0 * ts) + bo); };
#pragma unroll
  for (int c = 0; c < 10; c += 2) {
    const P2 v = ld(T_GCOV + c);
    g.gcov[c] = (T)v.x;
    g.gcov[c + 1] = (T)v.y;
  }
#pragma unroll
  for (int c = 0; c < 10; c += 2) {
    const P2 v = ld(T_GCON + c);
    g.gcon[c] = (T)v.x;
    g.gcon[c + 1] = (T)v.y;
  }
  const P2 v = ld(T_GDET);
  g.gdet = (T)v.x;
  g.alpha = (T)v.y;
}

// ---------------------------------------------------------------------------
// point physics (HARM variables; units GM = c = 1, b^2/2 magnetic pressure)

template <typename T>
struct Fluid {
  T ucon[4], ucov[4], bcon[4], bcov[4];
  T bsq, p, w;
};

template <typename T>
__device__ inline T lower(const T* gcov, const T* vcon, int m) {
  return gcov[sidx(m, 0)] * vcon[0] + gcov[sidx(m, 1)] * vcon[1] + gcov[sidx(m, 2)] * vcon[2] +
         gcov[sidx(m, 3)] * vcon[3];
}

// Gamma^2 = 1 + g_ij u~^i u~^j
template <typename T>
__device__ inline T lorentz_sq(const T* gcov, T v1, T v2, T v3) {
  return T(1) + gcov[4] * v1 * v1 + gcov[7] * v2 * v2 + gcov[9] * v3 * v3 +
         T(2) * (gcov[5] * v1 * v2 + gcov[6] * v1 * v3 + gcov[8] * v2 * v3);
}

// 1/sqrt(x) to full precision: the hardware estimate, then Newton steps
__device__ inline double rsqrt_full(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * (1.5 - 0.5 * x * r * r);
  return r * (1.5 - 0.5 * x * r * r);
}
__device__ inline float rsqrt_full(float x) {
  const float r = __builtin_amdgcn_rsqf(x);
  return r * (1.5f - 0.5f * x * r * r);
}

// the fluid four-vectors of primitives P. RSQ: Gamma and 1/u^t from one
// reciprocal square root (Gamma = G2 / sqrt(G2), 1/u^t = alpha / Gamma) instead
// of a square root and a division (the face-flux pass, where it is faster;
// the update keeps the plain form, whose register allocation it suits)
template <typename T, bool RSQ = false>
__device__ inline void fluid_state(const T* P, const Geo<T>& g, T gam, Fluid<T>& f) {
  const T l2 = lorentz_sq(g.gcov, P[2], P[3], P[4]);
  const T rl = RSQ ? rsqrt_full(l2) : T(0);
  const T lor = RSQ ? l2 * rl : sqrt(l2);
  f.ucon[0] = lor / g.alpha;
  const T la = lor * g.alpha;
  f.ucon[1] = P[2] - la * g.gcon[1];
  f.ucon[2] = P[3] - la * g.gcon[2];
  f.ucon[3] = P[4] - la * g.gcon[3];
#pragma unroll
  for (int m = 0; m < 4; ++m) f.ucov[m] = lower(g.gcov, f.ucon, m);
  const T bt = P[5] * f.ucov[1] + P[6] * f.ucov[2] + P[7] * f.ucov[3];
  const T iut = RSQ ? g.alpha * rl : T(1) / f.ucon[0];
  f.bcon[0] = bt;
  f.bcon[1] = (P[5] + bt * f.ucon[1]) * iut;
  f.bcon[2] = (P[6] + bt * f.ucon[2]) * iut;
  f.bcon[3] = (P[7] + bt * f.ucon[3]) * iut;
#pragma unroll
  for (int m = 0; m < 4; ++m) f.bcov[m] = lower(g.gcov, f.bcon, m);
  f.bsq = f.bcon[0] * f.bcov[0] + f.bcon[1] * f.bcov[1] + f.bcon[2] * f.bcov[2] + f.bcon[3] * f.bcov[3];
  f.p = (gam - T(1)) * P[1];
  f.w = P[0] + P[1] + f.p;
}

// sqrt(-g) F^D for D = 1..3, or U for D = 0 (B part sqrt(-g) B exactly).
// Energy component carries the rest-mass flux: T^D_t + rho u^D.
template <int D, typename T>
__device__ inline void flux_of(const T* P, const Fluid<T>& f, T gdet, T* F) {
  const T ud = f.ucon[D];
  const T mass = P[0] * ud;
  const T eb = (f.w + f.bsq) * ud;
  const T pt = f.p + T(0.5) * f.bsq;
  const T bd = f.bcon[D];
  F[0] = gdet * mass;
  F[1] = gdet * (eb * f.ucov[0] - bd * f.bcov[0] + (D == 0 ? pt : T(0)) + mass);
  F[2] = gdet * (eb * f.ucov[1] - bd * f.bcov[1] + (D == 1 ? pt : T(0)));
  F[3] = gdet * (eb * f.ucov[2] - bd * f.bcov[2] + (D == 2 ? pt : T(0)));
  F[4] = gdet * (eb * f.ucov[3] - bd * f.bcov[3] + (D == 3 ? pt : T(0)));
  if (D == 0) {
    F[5] = gdet * P[5];
    F[6] = gdet * P[6];
    F[7] = gdet * P[7];
  } else {
    F[5] = (D == 1) ? T(0) : gdet * (f.bcon[1] * ud - bd * f.ucon[1]);
    F[6] = (D == 2) ? T(0) : gdet * (f.bcon[2] * ud - bd * f.ucon[2]);
    F[7] = (D == 3) ? T(0) : gdet * (f.bcon[3] * ud - bd * f.ucon[3]);
  }
}

// Fast-magnetosonic speeds dx^D/dt: roots of A l^2 + B l + C = 0 with
// c^2 = v_A^2 + c_s^2 (1 - v_A^2), v_A^2 = b^2/(b^2 + w), c_s^2 = gamma p / w,
// which is the single quotient num/den = (b^2 + gamma p)/(b^2 + w); A, B and C
// are taken times den > 0, which leaves the roots unchanged and saves the
// division.
template <int D, typename T>
__device__ inline void signal_speeds(const Fluid<T>& f, const Geo<T>& g, T gam, T& cmax, T& cmin) {
  const T num = f.bsq + gam * f.p, den = f.bsq + f.w;
  const T ut = f.ucon[0], ud = f.ucon[D];
  const T A = den * ut * ut - num * (g.gcon[0] + ut * ut);
  const T B = T(-2) * (den * ut * ud - num * (g.gcon[D] + ut * ud));
  const T C = den * ud * ud - num * (g.gcon[sidx(D, D)] + ud * ud);
  const T disc = sqrt(fmax(B * B - T(4) * A * C, T(0)));
  const T i2a = T(1) / (T(2) * A);
  const T vp = (-B + disc) * i2a;
  const T vm = (-B - disc) * i2a;
  cmax = fmax(vp, vm);
  cmin = fmin(vp, vm);
}

// ---------------------------------------------------------------------------
// reconstruction

template <typename T>
__device__ inline T mc_slope(T pm, T p0, T pp) {
  const T dm = p0 - pm, dp = pp - p0, dc = T(0.5) * (pp - pm);
  // min(2|dm|, 2|dp|) = 2 min(|dm|, |dp|) exactly
  const T mag = fmin(T(2) * fmin(fabs(dm), fabs(dp)), fabs(dc));
  return (dm * dp > T(0)) ? copysign(mag, dc) : T(0);
}

// Value at the right edge of the middle zone of (x1..x5), point-value WENO5
// with Jiang-Shu smoothness indicators and linear weights (1/16, 5/8, 5/16):
// weights d_k / (eps + b_k)^2, normalised. Written over a common denominator,
// scaled by the smallest e_k = eps + b_k so nothing leaves the double range:
// with r_k = e_k / e_min >= 1, the weights are proportional to d_k times the
// product of the other two r_j^2 (two divisions instead of four).
__device__ inline double weno5_edge(double x1, double x2, double x3, double x4, double x5) {
  const double q0 = 0.375 * x1 - 1.25 * x2 + 1.875 * x3;
  const double q1 = -0.125 * x2 + 0.75 * x3 + 0.375 * x4;
  const double q2 = 0.375 * x3 + 0.75 * x4 - 0.125 * x5;
  const double t0 = x1 - 2.0 * x2 + x3, u0 = x1 - 4.0 * x2 + 3.0 * x3;
  const double t1 = x2 - 2.0 * x3 + x4, u1 = x2 - x4;
  const double t2 = x3 - 2.0 * x4 + x5, u2 = 3.0 * x3 - 4.0 * x4 + x5;
  const double e0 = 1e-26 + ((13.0 / 12.0) * t0 * t0 + 0.25 * u0 * u0);
  const double e1 = 1e-26 + ((13.0 / 12.0) * t1 * t1 + 0.25 * u1 * u1);
  const double e2 = 1e-26 + ((13.0 / 12.0) * t2 * t2 + 0.25 * u2 * u2);
  const double im = 1.0 / fmin(fmin(e0, e1), e2);
  // r_k <= 1e60 keeps the products of two squares finite; such a weight is 0 anyway
  const double r0 = fmin(e0 * im, 1e60), r1 = fmin(e1 * im, 1e60), r2 = fmin(e2 * im, 1e60);
  const double s0 = r0 * r0, s1 = r1 * r1, s2 = r2 * r2;
  const double a0 = 0.0625 * (s1 * s2), a1 = 0.625 * (s0 * s2), a2 = 0.3125 * (s0 * s1);
  return (a0 * q0 + a1 * q1 + a2 * q2) / (a0 + a1 + a2);
}

// FP32 form: eps^2 = 1e-52 is below the float range, so the weights use the
// ratios r_k = e_min / e_k in (0, 1]: d_k r_k^2, normalised; the term of the
// smallest e_k has r = 1, so the sum is at least 1/16. Reciprocals by the
// hardware rcp (about 1 ulp), far below the float rounding of the inputs.
__device__ inline float weno5_edge(float x1, float x2, float x3, float x4, float x5) {
  const float q0 = 0.375f * x1 - 1.25f * x2 + 1.875f * x3;
  const float q1 = -0.125f * x2 + 0.75f * x3 + 0.375f * x4;
  const float q2 = 0.375f * x3 + 0.75f * x4 - 0.125f * x5;
  const float t0 = x1 - 2.0f * x2 + x3, u0 = x1 - 4.0f * x2 + 3.0f * x3;
  const float t1 = x2 - 2.0f * x3 + x4, u1 = x2 - x4;
  const float t2 = x3 - 2.0f * x4 + x5, u2 = 3.0f * x3 - 4.0f * x4 + x5;
  const float e0 = 1e-26f + ((13.0f / 12.0f) * t0 * t0 + 0.25f * u0 * u0);
  const float e1 = 1e-26f + ((13.0f / 12.0f) * t1 * t1 + 0.25f * u1 * u1);
  const float e2 = 1e-26f + ((13.0f / 12.0f) * t2 * t2 + 0.25f * u2 * u2);
  const float m = fminf(fminf(e0, e1), e2);
  const float r0 = m * __builtin_amdgcn_rcpf(e0), r1 = m * __builtin_amdgcn_rcpf(e1),
              r2 = m * __builtin_amdgcn_rcpf(e2);
  const float a0 = 0.0625f * r0 * r0, a1 = 0.625f * r1 * r1, a2 = 0.3125f * r2 * r2;
  return (a0 * q0 + a1 * q1 + a2 * q2) * __builtin_amdgcn_rcpf(a0 + a1 + a2);
}

// ---------------------------------------------------------------------------
// XCD-aware block mapping
//
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Stencil kernels use a 1D grid of 8 * ntiles * chunk blocks, where a tile is
// a tx x ty (x1, x2) patch (one thread per cell, the block's shape) and
// chunk = ceil(nk / 8): XCD x receives, in order, every tile with k in
// [x*chunk, (x+1)*chunk). Consecutive blocks on one XCD then share the tile's
// 2D geometry and its neighbouring x3 planes in that XCD's L2 instead of
// refetching them once per x3 plane.

constexpr int NXCD = 8;
constexpr int TILE_X = 64;   // default tiles: face fluxes 64 x 8 (512 threads), update 64 x 1
constexpr int SWEEP_TILE_X = 64;
constexpr int SWEEP_TILE_Y = 8;
constexpr int TILE_Y = 1;
constexpr int SWEEP_MAX_THREADS = 512;   // launch bounds of the sweep kernels
constexpr int UPDATE_MAX_THREADS = 256;  // launch bounds of the update and fixup kernels

struct TileK {
  int i0, j0, k;
  bool valid;
};

// b: block index within this job's grid (a multiple-of-8 offset from the
// launch's block index, so b % 8 is still the XCD)
__device__ inline TileK xcd_tile_k(int b, int tx, int ty, int ni, int nk) {
  const int tiles_x = (ni + tx - 1) / tx;
  const int chunk = (nk + NXCD - 1) / NXCD;
  const int x = b % NXCD, w = b / NXCD;
  const int tile = w / chunk;
  TileK t;
  t.k = x * chunk + (w - tile * chunk);
  t.i0 = (tile % tiles_x) * tx;
  t.j0 = (tile / tiles_x) * ty;
  t.valid = t.k < nk;
  return t;
}

// 1D grid size for ni x nj x nk cells in tx x ty tiles
inline unsigned xcd_grid(int ni, int nj, int nk, int tx, int ty) {
  const int tiles = ((ni + tx - 1) / tx) * ((nj + ty - 1) / ty);
  const int chunk = (nk + NXCD - 1) / NXCD;
  return (unsigned)(NXCD * tiles * chunk);
}

// ---------------------------------------------------------------------------
// block reductions

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ inline int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// max of a non-negative double over the block, then one atomic max on the
// IEEE bit pattern (order-preserving for non-negative values). Callers map NaN
// to +inf first so a non-finite speed survives the reduction.
__device__ inline void block_max_to(double v, unsigned long long* dst) {
  __shared__ double part[16];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  v = wave_max(v + 0.0);
  if ((tid & 63) == 0) part[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    double m = part[0];
    for (int w = 1; w < (nthr + 63) / 64; ++w) m = fmax(m, part[w]);
    atomicMax(dst, (unsigned long long)__double_as_longlong(m + 0.0));
  }
}

// block_max_to for three values at once into dst[0..2]: one barrier, and
// the atomic only where the block's maximum exceeds the running one (values
// only grow, so a stale read can only cost an unneeded atomic)
__device__ inline void block_max3_to(double a, double b, double c, unsigned long long* dst) {
  __shared__ double part3[3][16];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  a = wave_max(a + 0.0);
  b = wave_max(b + 0.0);
  c = wave_max(c + 0.0);
  if ((tid & 63) == 0) {
    part3[0][tid >> 6] = a;
    part3[1][tid >> 6] = b;
    part3[2][tid >> 6] = c;
  }
  __syncthreads();
  if (tid < 3) {
    double m = part3[tid][0];
    for (int w = 1; w < (nthr + 63) / 64; ++w) m = fmax(m, part3[tid][w]);
    const unsigned long long bits = (unsigned long long)__double_as_longlong(m + 0.0);
    if (__hip_atomic_load(dst + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < bits) atomicMax(dst + tid, bits);
  }
}

// block sum of v, then one atomic add into dst (and into dst2 when given)
__device__ inline void block_count_to(int v, unsigned int* dst, unsigned int* dst2 = nullptr) {
  __shared__ int cpart[16];
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  v = wave_sum(v);
  if ((tid & 63) == 0) cpart[tid >> 6] = v;
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int w = 0; w < (nthr + 63) / 64; ++w) s += cpart[w];
    if (s) {
      atomicAdd(dst, (unsigned int)s);
      if (dst2) atomicAdd(dst2, (unsigned int)s);
    }
  }
}
