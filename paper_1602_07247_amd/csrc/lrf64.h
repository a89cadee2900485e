// FP64 evaluation of the LRFs on the device: uniform cubic B-splines on the
// extended knot vector (coefficient j centred on breakpoint j-1), value
// max(spline, 0) inside the domain (relative slack 1e-9 of the span) and 0
// outside.  Used for decisions, reported values and event generation.
#pragma once

#include "ants_internal.h"

namespace ants {
namespace {

// Interval m and local coordinate t of u on a uniform breakpoint grid
// (inv_d = 1 / spacing); false outside the domain (relative slack 1e-9).
__device__ __forceinline__ bool locate64(double u, int nb, double lo, double hi, double inv_d,
                                         int& m, double& t) {
  double tol = 1e-9 * (hi - lo);
  if (!(u >= lo - tol && u <= hi + tol)) return false;
  double v = (u - lo) * inv_d;
  int k = (int)floor(v);
  k = k < 0 ? 0 : k;
  k = k > nb - 2 ? nb - 2 : k;
  m = k;
  t = v - (double)k;
  return true;
}

// uniform cubic B-spline weights on one interval
__device__ __forceinline__ void bweights64(double t, double b[4]) {
  double s = 1.0 - t, t2 = t * t, t3 = t2 * t;
  b[0] = s * s * s * (1.0 / 6.0);
  b[1] = (3.0 * t3 - 6.0 * t2 + 4.0) * (1.0 / 6.0);
  b[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) * (1.0 / 6.0);
  b[3] = t3 * (1.0 / 6.0);
}

// Offset of a sensor's FP64 B-spline coefficients in c64 (composite: of
// its XY residual in xc64).
template <int KIND>
__device__ __forceinline__ int coef_off64(const DevLrf& L, int a) {
  if constexpr (KIND == ANTS_LRF_AXIAL) return L.tab[a] * L.nc0;
  else if constexpr (KIND == ANTS_LRF_XY) return L.tab[a] * L.nc0 * L.nc1;
  else if constexpr (KIND == ANTS_LRF_COMPOSITE) return L.xtab[a] * L.xnc0 * L.xnc1;
  else if constexpr (KIND == ANTS_LRF_SLICED) return L.tab[a] * L.nplanes * L.nc0 * L.nc1;
  else return 0;
}

// FP64 bicubic B-spline (table [nc1][nc0]) at (u, w); 0 outside the domain
__device__ __forceinline__ double spline2_64(const double* c, int nc0, int nb0, int nb1,
                                             double lo0, double hi0, double lo1, double hi1,
                                             double inv_d0, double inv_d1, double u, double w) {
  int m0, m1;
  double t0, t1, b0[4], b1[4];
  if (!locate64(u, nb0, lo0, hi0, inv_d0, m0, t0)) return 0.0;
  if (!locate64(w, nb1, lo1, hi1, inv_d1, m1, t1)) return 0.0;
  bweights64(t0, b0);
  bweights64(t1, b1);
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double* row = c + (size_t)(m1 + q) * nc0 + m0;
    v += b1[q] * (row[0] * b0[0] + row[1] * b0[1] + row[2] * b0[2] + row[3] * b0[3]);
  }
  return v;
}

// FP64 LRF at (x, y, z) of a sensor at (X, Y) whose coefficients start at
// c64 + coff.
template <int KIND>
__device__ __forceinline__ double lrf64s(const DevLrf& L, double X, double Y, int coff, double x,
                                         double y, double z) {
  double v = 0.0;
  if constexpr (KIND == ANTS_LRF_COMPOSITE) {
    // axial part (one shared row) plus the XY residual, each 0 outside its
    // domain, the sum clamped
    double dx = x - X, dy = y - Y;
    double r = sqrt(dx * dx + dy * dy);
    int m;
    double t, b[4];
    if (locate64(r, L.nb0, L.lo0, L.hi0, L.inv_d0, m, t)) {
      bweights64(t, b);
      const double* c = L.c64 + m;
      v = c[0] * b[0] + c[1] * b[1] + c[2] * b[2] + c[3] * b[3];
    }
    v += spline2_64(L.xc64 + coff, L.xnc0, L.xnb0, L.xnb1, L.xlo0, L.xhi0, L.xlo1, L.xhi1,
                    L.xinv_d0, L.xinv_d1, x, y);
    return v > 0.0 ? v : 0.0;
  } else if constexpr (KIND == ANTS_LRF_SLICED) {
    // the two closest planes' clamped XY values, linear in z between them
    int p;
    double t;
    if (!locate64(z, L.nplanes, L.zlo, L.zhi, L.inv_dz, p, t)) return 0.0;
    const int plane = L.nc0 * L.nc1;
    double a = spline2_64(L.c64 + coff + p * plane, L.nc0, L.nb0, L.nb1, L.lo0, L.hi0, L.lo1,
                          L.hi1, L.inv_d0, L.inv_d1, x, y);
    double b = spline2_64(L.c64 + coff + (p + 1) * plane, L.nc0, L.nb0, L.nb1, L.lo0, L.hi0,
                          L.lo1, L.hi1, L.inv_d0, L.inv_d1, x, y);
    a = a > 0.0 ? a : 0.0;
    b = b > 0.0 ? b : 0.0;
    return (1.0 - t) * a + t * b;
  } else if constexpr (KIND == ANTS_LRF_AXIAL) {
    double dx = x - X, dy = y - Y;
    double r = sqrt(dx * dx + dy * dy);
    int m;
    double t, b[4];
    if (!locate64(r, L.nb0, L.lo0, L.hi0, L.inv_d0, m, t)) return 0.0;
    bweights64(t, b);
    const double* c = L.c64 + coff + m;
    v = c[0] * b[0] + c[1] * b[1] + c[2] * b[2] + c[3] * b[3];
  } else {
    double u, w;
    const double* c = L.c64 + coff;
    if constexpr (KIND == ANTS_LRF_RZ) {
      double dx = x - X, dy = y - Y;
      u = sqrt(dx * dx + dy * dy);
      w = z;
    } else {
      u = x;
      w = y;
    }
    int m0, m1;
    double t0, t1, b0[4], b1[4];
    if (!locate64(u, L.nb0, L.lo0, L.hi0, L.inv_d0, m0, t0)) return 0.0;
    if (!locate64(w, L.nb1, L.lo1, L.hi1, L.inv_d1, m1, t1)) return 0.0;
    bweights64(t0, b0);
    bweights64(t1, b1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double* row = c + (size_t)(m1 + q) * L.nc0 + m0;
      v += b1[q] * (row[0] * b0[0] + row[1] * b0[1] + row[2] * b0[2] + row[3] * b0[3]);
    }
  }
  return v > 0.0 ? v : 0.0;
}
template <int KIND>
__device__ __forceinline__ double lrf64(const DevLrf& L, int a, double x, double y, double z) {
  return lrf64s<KIND>(L, L.X[a], L.Y[a], coef_off64<KIND>(L, a), x, y, z);
}

__device__ __forceinline__ bool in_domain(double u, double lo, double hi) {
  double tol = 1e-9 * (hi - lo);
  return u >= lo - tol && u <= hi + tol;
}

}  // namespace
}  // namespace ants
