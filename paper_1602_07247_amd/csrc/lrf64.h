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

// Offset of a sensor's FP64 B-spline coefficients in c64.
template <int KIND>
__device__ __forceinline__ int coef_off64(const DevLrf& L, int a) {
  if constexpr (KIND == ANTS_LRF_AXIAL) return L.tab[a] * L.nc0;
  else if constexpr (KIND == ANTS_LRF_XY) return L.tab[a] * L.nc0 * L.nc1;
  else return 0;
}

// FP64 LRF at (x, y, z) of a sensor at (X, Y) whose coefficients start at
// c64 + coff.
template <int KIND>
__device__ __forceinline__ double lrf64s(const DevLrf& L, double X, double Y, int coff, double x,
                                         double y, double z) {
  double v = 0.0;
  if constexpr (KIND == ANTS_LRF_AXIAL) {
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
