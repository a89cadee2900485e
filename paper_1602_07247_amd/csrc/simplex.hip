// Simplex search per event (Sec. 5.1.2.1: the Minuit2 Simplex minimiser
// over x, y or x, y, z, started at the centroid or the strongest sensor),
// as the Nelder-Mead method of Lagarias, Reeds, Wright and Wright (SIAM J.
// Optim. 9, 1998) with coefficients 1 (reflection), 2 (expansion), 1/2
// (contraction) and 1/2 (shrink).  The energy is the ratio of the sums
// (Sec. 5.1.2.2) at every point, so only the position is searched.
//
// Mapping: one wavefront per event; every point of the search is evaluated
// in FP64 with lanes over the active sensors and a wave sum.  Every value
// the method compares is FP64, and values within 1e-12 N of each other are
// equal (the grid's tie rule): vertices stay ordered by value with a new
// vertex placed after those equal to it.  Vertex coordinates are computed
// as written (no fused multiply-add) so the trial points are those of the
// FP64 definition.
#include <math.h>

#include "ants_internal.h"
#include "lrf64.h"

namespace ants {
namespace {

constexpr double kTieRelSx = 1e-12;   // tie tolerance, relative to N

__device__ __forceinline__ double wsum64(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

struct SxP {
  DevLrf L;
  int dims, stat, start, max_iter;
  double s0[3], z_start, tol, lfloor, vfloor;
  double h, edm;        // variable-metric search: difference step, EDM tolerance
  IoP io;
  int32_t* iters;
};

struct Vtx {
  double x, y, z, f;
};

// Statistic at (x, y, z): ML N ln S - sum n ln max(L, l_floor) (the
// negative log-likelihood up to a constant of the event), or chi2; +inf
// when S <= 0.
template <int KIND, int STAT, int SL>
__device__ __forceinline__ double sx_eval(const SxP& P, const float (&nq)[SL], double N, double x,
                                          double y, double z, int lane) {
  const DevLrf& L = P.L;
  double S = 0.0, T = 0.0, Lv[SL];
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int a = lane + 64 * q;
    Lv[q] = 0.0;
    if (a < L.na) {
      Lv[q] = lrf64<KIND>(L, a, x, y, z);
      S += L.g[a] * Lv[q];
      if (STAT == ANTS_STAT_ML && nq[q] > 0.f)
        T += (double)nq[q] * log(Lv[q] > P.lfloor ? Lv[q] : P.lfloor);
    }
  }
  S = wsum64(S);
  if (!(S > 0.0) || !(S < __builtin_huge_val())) return __builtin_huge_val();
  double f;
  if constexpr (STAT == ANTS_STAT_ML) {
    f = N * log(S) - wsum64(T);
  } else {
    const double A = N / S;
    double Q = 0.0;
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      const int a = lane + 64 * q;
      if (a < L.na) {
        const double mu = A * L.g[a] * Lv[q];
        const double dd = (double)nq[q] - mu;
        Q += dd * dd / (mu > P.vfloor ? mu : P.vfloor);
      }
    }
    f = wsum64(Q);
  }
  return f < __builtin_huge_val() ? f : __builtin_huge_val();
}

__device__ __forceinline__ bool lt(double a, double b, double tol) { return a < b - tol; }

// insert w after every vertex of v[0..n-1] whose value is not above w's
// (w placed at n, then moved down past the vertices it is below; compile-
// time indices keep the vertices in registers)
template <int n>
__device__ __forceinline__ void sx_insert(Vtx (&v)[4], const Vtx& w, double tol) {
  v[n] = w;
#pragma unroll
  for (int i = n; i > 0; --i) {
    if (!lt(v[i].f, v[i - 1].f, tol)) break;
    const Vtx t = v[i];
    v[i] = v[i - 1];
    v[i - 1] = t;
  }
}

// Event set-up shared by the searches: signals of the active sensors, N,
// status (NaN outputs written for a failed event; returns false) and the
// start (Sec. 5.1.1 centroid, Sec. 5.1.2.1 strongest sensor, or seed).
template <int SL, int D>
__device__ __forceinline__ bool search_start(const SxP& P, int64_t e, int lane, float (&nq)[SL],
                                             double& N, double (&c0)[3]) {
  const DevLrf& L = P.L;
  const IoP& io = P.io;
  const float* row = io.sig + e * io.ld;
  const int na = L.na;
  constexpr int d = D;
  N = 0.0;
  double cw = 0.0, cxs = 0.0, cys = 0.0;
  bool bad = false;
  float best_n = -1.0f;
  int best_a = 1 << 30;
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int a = lane + 64 * q;
    nq[q] = 0.f;
    if (a < na) {
      const float n = row[L.col[a]];
      nq[q] = n;
      if (!(n >= 0.f) || !(n < __builtin_huge_valf())) {
        bad = true;
      } else {
        N += (double)n;
        const double w = (double)n / L.g[a];
        cw += w;
        cxs += L.X[a] * w;
        cys += L.Y[a] * w;
        if (n > best_n || (n == best_n && a < best_a)) {
          best_n = n;
          best_a = a;
        }
      }
    }
  }
  const bool any_bad = __ballot(bad) != 0ull;
  N = wsum64(N);
  const int ndf = na - (d + 1);
  const int status = na == 0 ? ANTS_EV_NO_ACTIVE : any_bad ? ANTS_EV_BAD_INPUT
                     : !(N > 0.0)                ? ANTS_EV_EMPTY
                                                 : 0;
  if (status) {
    if (lane == 0) {
      const float nan = __builtin_nanf("");
      io.x[e] = nan; io.y[e] = nan; io.z[e] = nan; io.E[e] = nan;
      io.lnl[e] = nan; io.chi2[e] = nan; io.ndf[e] = ndf; io.status[e] = status;
      if (P.iters) P.iters[e] = 0;
      if (io.nfp) io.nfp[e] = 0;
    }
    return false;
  }
  c0[0] = 0.0;
  c0[1] = 0.0;
  c0[2] = P.z_start;
  if (P.start == ANTS_START_SEED && io.seeds) {
    c0[0] = io.seeds[e * 4 + 0];
    c0[1] = io.seeds[e * 4 + 1];
    if (d == 3) c0[2] = io.seeds[e * 4 + 2];
  } else if (P.start == ANTS_START_MAXSENSOR) {
    // strongest sensor, lowest index on ties
    for (int o = 32; o >= 1; o >>= 1) {
      const float n2 = __shfl_xor(best_n, o);
      const int a2 = __shfl_xor(best_a, o);
      if (n2 > best_n || (n2 == best_n && a2 < best_a)) {
        best_n = n2;
        best_a = a2;
      }
    }
    c0[0] = L.X[best_a];
    c0[1] = L.Y[best_a];
  } else {
    cw = wsum64(cw);
    c0[0] = wsum64(cxs) / cw;
    c0[1] = wsum64(cys) / cw;
  }
  return true;
}

// Outputs at the final point (x, y, z), FP64, lane-parallel over sensors.
template <int KIND, int SL>
__device__ __forceinline__ void search_outputs(const SxP& P, int64_t e, int lane,
                                               const float (&nq)[SL], double N, double bx,
                                               double by, double bz, int d, int status, int it,
                                               int nev) {
#pragma clang fp contract(off)
  const DevLrf& L = P.L;
  const IoP& io = P.io;
  const int na = L.na;
  double S = 0.0, Lf[SL];
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int a = lane + 64 * q;
    Lf[q] = 0.0;
    if (a < na) {
      Lf[q] = lrf64<KIND>(L, a, bx, by, bz);
      S += L.g[a] * Lf[q];
    }
  }
  S = wsum64(S);
  const bool okS = S > 0.0 && S < __builtin_huge_val();
  double Aa = N / S, ll = 0.0, q2 = 0.0;
  if (okS) {
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      const int a = lane + 64 * q;
      if (a < na) {
        const double mu = Aa * L.g[a] * Lf[q];
        const double Lt = Lf[q] > P.lfloor ? Lf[q] : P.lfloor;
        const double n = (double)nq[q];
        if (n > 0.0) ll += n * log(Aa * L.g[a] * Lt);
        ll -= mu;
        const double dd = n - mu;
        q2 += dd * dd / (mu > P.vfloor ? mu : P.vfloor);
      }
    }
    ll = wsum64(ll);
    q2 = wsum64(q2);
  } else {
    status |= ANTS_EV_NO_VALID_NODE;
  }
  if (lane == 0) {
    const float nan = __builtin_nanf("");
    io.x[e] = (float)bx;
    io.y[e] = (float)by;
    io.z[e] = (float)bz;
    io.E[e] = okS ? (float)Aa : nan;
    io.lnl[e] = okS ? (float)ll : nan;
    io.chi2[e] = okS ? (float)q2 : nan;
    io.ndf[e] = na - (d + 1);
    io.status[e] = status;
    if (P.iters) P.iters[e] = it;
    if (io.nfp) io.nfp[e] = nev;
  }
}

template <int KIND, int STAT, int SL, int D>
__device__ void sx_event(const SxP& P, int64_t e, int lane) {
#pragma clang fp contract(off)
  constexpr int d = D;
  float nq[SL];
  double N, c0[3];
  if (!search_start<SL, D>(P, e, lane, nq, N, c0)) return;
  int status = 0;
  const double tf = kTieRelSx * N;
  Vtx v[4];
  {
    Vtx w[4];
#pragma unroll
    for (int i = 0; i <= d; ++i) {
      w[i] = Vtx{c0[0], c0[1], c0[2], 0.0};
      if (i == 1) w[i].x = c0[0] + P.s0[0];
      if (i == 2) w[i].y = c0[1] + P.s0[1];
      if (i == 3) w[i].z = c0[2] + P.s0[2];
      w[i].f = sx_eval<KIND, STAT, SL>(P, nq, N, w[i].x, w[i].y, w[i].z, lane);
    }
    v[0] = w[0];
    sx_insert<1>(v, w[1], tf);
    sx_insert<2>(v, w[2], tf);
    if constexpr (d == 3) sx_insert<3>(v, w[3], tf);
  }
  int it = 0, nev = d + 1;
  for (;;) {
    bool conv = true;
#pragma unroll
    for (int i = 1; i <= d; ++i) {
      conv = conv && fabs(v[i].x - v[0].x) <= P.tol && fabs(v[i].y - v[0].y) <= P.tol;
      if (d == 3) conv = conv && fabs(v[i].z - v[0].z) <= P.tol;
    }
    if (conv) break;
    if (!(v[0].f < __builtin_huge_val())) {
      status |= ANTS_EV_NO_VALID_NODE;
      break;
    }
    if (it >= P.max_iter) break;
    ++it;
    // centroid of the d best vertices (sum in vertex order, then divide)
    double cx = 0.0, cy = 0.0, cz = 0.0;
#pragma unroll
    for (int i = 0; i < d; ++i) {
      cx += v[i].x;
      cy += v[i].y;
      cz += v[i].z;
    }
    cx = cx / (double)d;
    cy = cy / (double)d;
    cz = d == 3 ? cz / (double)d : v[0].z;
    const Vtx& wv = v[d];
    Vtx r{cx + (cx - wv.x), cy + (cy - wv.y), d == 3 ? cz + (cz - wv.z) : cz, 0.0};
    r.f = sx_eval<KIND, STAT, SL>(P, nq, N, r.x, r.y, r.z, lane);
    ++nev;
    Vtx acc = r;
    bool shrink = false;
    if (!lt(r.f, v[0].f, tf) && lt(r.f, v[d - 1].f, tf)) {
      acc = r;                                            // reflection
    } else if (lt(r.f, v[0].f, tf)) {
      Vtx x{cx + 2.0 * (r.x - cx), cy + 2.0 * (r.y - cy), d == 3 ? cz + 2.0 * (r.z - cz) : cz,
            0.0};                                         // expansion
      x.f = sx_eval<KIND, STAT, SL>(P, nq, N, x.x, x.y, x.z, lane);
      ++nev;
      acc = lt(x.f, r.f, tf) ? x : r;
    } else if (lt(r.f, wv.f, tf)) {
      Vtx k{cx + 0.5 * (r.x - cx), cy + 0.5 * (r.y - cy), d == 3 ? cz + 0.5 * (r.z - cz) : cz,
            0.0};                                         // outside contraction
      k.f = sx_eval<KIND, STAT, SL>(P, nq, N, k.x, k.y, k.z, lane);
      ++nev;
      if (!lt(r.f, k.f, tf)) acc = k;
      else shrink = true;
    } else {
      Vtx k{cx + 0.5 * (wv.x - cx), cy + 0.5 * (wv.y - cy),
            d == 3 ? cz + 0.5 * (wv.z - cz) : cz, 0.0};  // inside contraction
      k.f = sx_eval<KIND, STAT, SL>(P, nq, N, k.x, k.y, k.z, lane);
      ++nev;
      if (lt(k.f, wv.f, tf)) acc = k;
      else shrink = true;
    }
    if (!shrink) {
      sx_insert<d>(v, acc, tf);
    } else {
      Vtx w[4];
#pragma unroll
      for (int i = 1; i <= d; ++i) {
        w[i].x = v[0].x + 0.5 * (v[i].x - v[0].x);
        w[i].y = v[0].y + 0.5 * (v[i].y - v[0].y);
        w[i].z = d == 3 ? v[0].z + 0.5 * (v[i].z - v[0].z) : v[0].z;
        w[i].f = sx_eval<KIND, STAT, SL>(P, nq, N, w[i].x, w[i].y, w[i].z, lane);
      }
      nev += d;
      // the best vertex stays first; the others re-enter in order
      sx_insert<1>(v, w[1], tf);
      sx_insert<2>(v, w[2], tf);
      if constexpr (d == 3) sx_insert<3>(v, w[3], tf);
    }
  }
  search_outputs<KIND, SL>(P, e, lane, nq, N, v[0].x, v[0].y, v[0].z, d, status, it, nev);
}

// Variable-metric search (Sec. 5.1.2.1: the Minuit2 Migrad minimiser, a
// variable-metric method with numerical derivatives): central-difference
// gradients with step h, an initial diagonal inverse curvature from the
// same differences (step0^2 where it is not positive), direction -V g, a
// halving line search with the Armijo condition (factor 1e-4, at most 20
// halvings), the BFGS update of V when s^T y > 0, and a stop when EDM =
// g^T V g / 2 falls below the tolerance.  Coordinates that are arguments
// of the LRF's splines (z of r-z and sliced LRFs, x and y of XY and sliced
// LRFs) are limited to the spline's domain as Minuit limits parameters:
// the search runs in u with the position lo + (hi - lo) (sin u + 1) / 2.
// Every value is the FP64 statistic of the wave (identical in every
// lane); arithmetic as written (no fused multiply-add), sums in axis order.
template <int KIND, int STAT, int SL, int D>
__device__ void vm_event(const SxP& P, int64_t e, int lane) {
#pragma clang fp contract(off)
  constexpr int d = D;
  float nq[SL];
  double N, p[3];
  if (!search_start<SL, D>(P, e, lane, nq, N, p)) return;
  const DevLrf& L = P.L;
  // limited axes: lower end and half width of the spline domain
  bool lim[3] = {false, false, false};
  double llo[3] = {0.0, 0.0, 0.0}, lhalf[3] = {1.0, 1.0, 1.0};
  if constexpr (KIND == ANTS_LRF_XY || KIND == ANTS_LRF_SLICED) {
    lim[0] = lim[1] = true;
    llo[0] = L.lo0;
    lhalf[0] = 0.5 * (L.hi0 - L.lo0);
    llo[1] = L.lo1;
    lhalf[1] = 0.5 * (L.hi1 - L.lo1);
  }
  if constexpr (d == 3 && (KIND == ANTS_LRF_RZ || KIND == ANTS_LRF_SLICED)) {
    const double zl = KIND == ANTS_LRF_RZ ? L.lo1 : L.zlo, zh = KIND == ANTS_LRF_RZ ? L.hi1 : L.zhi;
    lim[2] = true;
    llo[2] = zl;
    lhalf[2] = 0.5 * (zh - zl);
  }
  // internal coordinates, difference steps and fallback scales
  double u[3] = {p[0], p[1], p[2]}, hs[3], s0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    hs[a] = P.h;
    s0[a] = P.s0[a];
  }
#pragma unroll
  for (int a = 0; a < d; ++a) {
    if (!lim[a]) continue;
    double w = (p[a] - llo[a]) / lhalf[a] - 1.0;
    w = w < -1.0 ? -1.0 : w > 1.0 ? 1.0 : w;
    u[a] = asin(w);
    hs[a] = P.h / lhalf[a];
    s0[a] = P.s0[a] / lhalf[a];
  }
  int nev = 0, it = 0;
  // statistic at internal point q
  auto F = [&](const double (&q)[3]) -> double {
    ++nev;
    double x[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      x[a] = (a < d && lim[a]) ? llo[a] + lhalf[a] * (sin(q[a]) + 1.0) : q[a];
    return sx_eval<KIND, STAT, SL>(P, nq, N, x[0], x[1], d == 3 ? x[2] : P.z_start, lane);
  };
  // central differences at q (F(q) = fq): gradient and curvature estimates
  auto grad = [&](const double (&q)[3], double fq, double (&g)[3], double (&d2)[3]) -> bool {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      g[a] = 0.0;
      d2[a] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < d; ++a) {
      double qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
      qp[a] = q[a] + hs[a];
      qm[a] = q[a] - hs[a];
      const double fp = F(qp);
      const double fm = F(qm);
      if (!(fp < __builtin_huge_val()) || !(fm < __builtin_huge_val())) ok = false;
      g[a] = (fp - fm) / (2.0 * hs[a]);
      d2[a] = ((fp - 2.0 * fq) + fm) / (hs[a] * hs[a]);
      if (!ok) break;
    }
    return ok;
  };
  double f = F(u);
  double g[3], d2[3], V[3][3];
  if (f < __builtin_huge_val() && grad(u, f, g, d2)) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) V[a][b] = 0.0;
#pragma unroll
    for (int a = 0; a < d; ++a)
      V[a][a] = (d2[a] > 0.0 && d2[a] < __builtin_huge_val()) ? 1.0 / d2[a] : s0[a] * s0[a];
    while (it < P.max_iter) {
      double Vg[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < d; ++a)
#pragma unroll
        for (int b = 0; b < d; ++b) Vg[a] += V[a][b] * g[b];
      double edm = 0.0;
#pragma unroll
      for (int a = 0; a < d; ++a) edm += g[a] * Vg[a];
      edm = 0.5 * edm;
      if (edm < P.edm) break;
      double dir[3] = {0.0, 0.0, 0.0}, slope = 0.0;
#pragma unroll
      for (int a = 0; a < d; ++a) {
        dir[a] = -Vg[a];
        slope += g[a] * dir[a];
      }
      if (!(slope < 0.0)) {
#pragma unroll
        for (int a = 0; a < d; ++a)
#pragma unroll
          for (int b = 0; b < d; ++b) V[a][b] = (a == b) ? s0[a] * s0[a] : 0.0;
        slope = 0.0;
#pragma unroll
        for (int a = 0; a < d; ++a) {
          dir[a] = -(V[a][a] * g[a]);
          slope += g[a] * dir[a];
        }
        if (!(slope < 0.0)) break;
      }
      double alpha = 1.0, pt[3] = {u[0], u[1], u[2]}, ft = __builtin_huge_val();
      bool ok = false;
      for (int ls = 0; ls <= 20; ++ls) {
#pragma unroll
        for (int a = 0; a < d; ++a) pt[a] = u[a] + alpha * dir[a];
        ft = F(pt);
        if (ft <= f + 1e-4 * alpha * slope) {
          ok = true;
          break;
        }
        alpha = 0.5 * alpha;
      }
      if (!ok) break;
      double gn[3], d2n[3];
      const bool gok = grad(pt, ft, gn, d2n);
      double sv[3] = {0.0, 0.0, 0.0}, yv[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < d; ++a) {
        sv[a] = pt[a] - u[a];
        yv[a] = gn[a] - g[a];
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) u[a] = pt[a];
      f = ft;
      ++it;
      if (!gok) break;
      double sy = 0.0;
#pragma unroll
      for (int a = 0; a < d; ++a) sy += sv[a] * yv[a];
      if (sy > 0.0) {
        double Vy[3] = {0.0, 0.0, 0.0}, yVy = 0.0;
#pragma unroll
        for (int a = 0; a < d; ++a)
#pragma unroll
          for (int b = 0; b < d; ++b) Vy[a] += V[a][b] * yv[b];
#pragma unroll
        for (int a = 0; a < d; ++a) yVy += yv[a] * Vy[a];
        const double c1 = (sy + yVy) / (sy * sy);
#pragma unroll
        for (int a = 0; a < d; ++a)
#pragma unroll
          for (int b = 0; b < d; ++b)
            V[a][b] = (V[a][b] + c1 * (sv[a] * sv[b])) - (Vy[a] * sv[b] + sv[a] * Vy[b]) / sy;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) g[a] = gn[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    p[a] = (a < d && lim[a]) ? llo[a] + lhalf[a] * (sin(u[a]) + 1.0) : u[a];
  if (d == 2) p[2] = P.z_start;
  const int status = f < __builtin_huge_val() ? 0 : ANTS_EV_NO_VALID_NODE;
  search_outputs<KIND, SL>(P, e, lane, nq, N, p[0], p[1], p[2], d, status, it, nev);
}

template <int KIND, int STAT, int SL, int D>
__global__ void __launch_bounds__(256) migrad_kernel(SxP P) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w0 = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t stride = (int64_t)gridDim.x * wpb;
  for (int64_t e = w0; e < P.io.n; e += stride) vm_event<KIND, STAT, SL, D>(P, e, lane);
}

template <int KIND, int STAT, int SL, int D>
__global__ void __launch_bounds__(256) simplex_kernel(SxP P) {
  const int lane = threadIdx.x & 63;
  const int64_t wpb = blockDim.x >> 6;
  const int64_t w0 = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6);
  const int64_t stride = (int64_t)gridDim.x * wpb;
  for (int64_t e = w0; e < P.io.n; e += stride) sx_event<KIND, STAT, SL, D>(P, e, lane);
}

// VM: the variable-metric search instead of the simplex
template <int KIND, int STAT, int SL, bool VM>
hipError_t launch_sx_kss(const SxP& P, int blocks, hipStream_t s) {
  const bool d3 = (KIND == ANTS_LRF_RZ || KIND == ANTS_LRF_SLICED) && P.dims == 3;
  if constexpr (VM) {
    if (d3) hipLaunchKernelGGL((migrad_kernel<KIND, STAT, SL, 3>), dim3(blocks), dim3(256), 0, s, P);
    else hipLaunchKernelGGL((migrad_kernel<KIND, STAT, SL, 2>), dim3(blocks), dim3(256), 0, s, P);
  } else {
    if (d3) hipLaunchKernelGGL((simplex_kernel<KIND, STAT, SL, 3>), dim3(blocks), dim3(256), 0, s, P);
    else hipLaunchKernelGGL((simplex_kernel<KIND, STAT, SL, 2>), dim3(blocks), dim3(256), 0, s, P);
  }
  return hipGetLastError();
}

template <int KIND, int STAT, bool VM>
hipError_t launch_sx_ks(const SxP& P, int blocks, hipStream_t s) {
  if (P.L.na <= 64) return launch_sx_kss<KIND, STAT, 1, VM>(P, blocks, s);
  if (P.L.na <= 128) return launch_sx_kss<KIND, STAT, 2, VM>(P, blocks, s);
  return launch_sx_kss<KIND, STAT, 4, VM>(P, blocks, s);
}

template <int KIND, bool VM>
hipError_t launch_sx_k(const SxP& P, int blocks, hipStream_t s) {
  return P.stat == ANTS_STAT_ML ? launch_sx_ks<KIND, ANTS_STAT_ML, VM>(P, blocks, s)
                                : launch_sx_ks<KIND, ANTS_STAT_CHI2, VM>(P, blocks, s);
}

template <bool VM>
hipError_t launch_search(const SxP& P, int blocks, hipStream_t s) {
  const int k = P.L.kind;
  return k == ANTS_LRF_AXIAL       ? launch_sx_k<ANTS_LRF_AXIAL, VM>(P, blocks, s)
         : k == ANTS_LRF_XY        ? launch_sx_k<ANTS_LRF_XY, VM>(P, blocks, s)
         : k == ANTS_LRF_COMPOSITE ? launch_sx_k<ANTS_LRF_COMPOSITE, VM>(P, blocks, s)
         : k == ANTS_LRF_SLICED    ? launch_sx_k<ANTS_LRF_SLICED, VM>(P, blocks, s)
                                   : launch_sx_k<ANTS_LRF_RZ, VM>(P, blocks, s);
}

}  // namespace
}  // namespace ants

using namespace ants;

extern "C" ants_status ants_reconstruct_simplex(ants_lrfset* set, const ants_simplex_cfg* cfg,
                                                int64_t n_events, const float* d_signals,
                                                const float* d_seeds, ants_out out,
                                                int32_t* d_iters, void* hip_stream) {
  if (!set || !cfg) return set_error(ANTS_E_ARG, "ants_reconstruct_simplex: NULL set or cfg");
  if (n_events < 0 || n_events > ((int64_t)1 << 31) - 1)
    return set_error(ANTS_E_ARG, "n_events = %lld out of range", (long long)n_events);
  const DevLrf& L = set->d;
  if (cfg->dims != 2 && cfg->dims != 3)
    return set_error(ANTS_E_ARG, "dims = %d must be 2 or 3", cfg->dims);
  if (cfg->dims == 3 && L.kind != ANTS_LRF_RZ && L.kind != ANTS_LRF_SLICED)
    return set_error(ANTS_E_ARG, "a 3-D search needs an r-z or sliced LRF");
  if (cfg->stat != ANTS_STAT_ML && cfg->stat != ANTS_STAT_CHI2)
    return set_error(ANTS_E_ARG, "unknown statistic %d", cfg->stat);
  if (cfg->start < ANTS_START_COG || cfg->start > ANTS_START_SEED)
    return set_error(ANTS_E_ARG, "unknown start option %d", cfg->start);
  if (cfg->start == ANTS_START_SEED && !d_seeds && n_events > 0)
    return set_error(ANTS_E_ARG, "start = SEED needs d_seeds");
  for (int a = 0; a < cfg->dims; ++a)
    if (!(cfg->step0[a] > 0.0 && isfinite(cfg->step0[a])))
      return set_error(ANTS_E_ARG, "step0[%d] = %g must be positive", a, cfg->step0[a]);
  if (!(cfg->tol > 0.0 && isfinite(cfg->tol)))
    return set_error(ANTS_E_ARG, "tol = %g must be positive", cfg->tol);
  if (cfg->max_iter < 0 || cfg->max_iter > 100000)
    return set_error(ANTS_E_ARG, "max_iter = %d outside 0..100000", cfg->max_iter);
  if (!(cfg->l_floor > 0.0) || !(cfg->v_floor > 0.0))
    return set_error(ANTS_E_ARG, "l_floor and v_floor must be positive");
  if (!isfinite(cfg->z_start)) return set_error(ANTS_E_ARG, "z_start not finite");
  if (n_events == 0) return ANTS_OK;
  if (!d_signals || !out.x || !out.y || !out.z || !out.E || !out.lnl || !out.chi2 || !out.ndf ||
      !out.status)
    return set_error(ANTS_E_ARG, "NULL signal or output pointer");
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != set->device) return set_error(ANTS_E_ARG, "LRF set lives on another device");
  SxP P;
  P = SxP{};
  P.L = L;
  P.dims = cfg->dims;
  P.stat = cfg->stat;
  P.start = cfg->start;
  P.max_iter = cfg->max_iter;
  for (int a = 0; a < 3; ++a) P.s0[a] = a < cfg->dims ? cfg->step0[a] : 0.0;
  P.z_start = cfg->z_start;
  P.tol = cfg->tol;
  P.lfloor = cfg->l_floor;
  P.vfloor = cfg->v_floor;
  P.io.sig = d_signals;
  P.io.ld = set->ns;
  P.io.seeds = cfg->start == ANTS_START_SEED ? d_seeds : nullptr;
  P.io.x = out.x;
  P.io.y = out.y;
  P.io.z = out.z;
  P.io.E = out.E;
  P.io.lnl = out.lnl;
  P.io.chi2 = out.chi2;
  P.io.ndf = out.ndf;
  P.io.status = out.status;
  P.io.nfp = out.n_fp64;
  P.io.n = n_events;
  P.iters = d_iters;
  int64_t blocks = (n_events + 3) / 4;
  const int64_t cap = (int64_t)num_cu() * 16;
  if (blocks > cap) blocks = cap;
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = launch_search<false>(P, (int)blocks, s);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_reconstruct_simplex launch");
}

extern "C" ants_status ants_reconstruct_migrad(ants_lrfset* set, const ants_migrad_cfg* cfg,
                                               int64_t n_events, const float* d_signals,
                                               const float* d_seeds, ants_out out,
                                               int32_t* d_iters, void* hip_stream) {
  if (!set || !cfg) return set_error(ANTS_E_ARG, "ants_reconstruct_migrad: NULL set or cfg");
  if (n_events < 0 || n_events > ((int64_t)1 << 31) - 1)
    return set_error(ANTS_E_ARG, "n_events = %lld out of range", (long long)n_events);
  const DevLrf& L = set->d;
  if (cfg->dims != 2 && cfg->dims != 3)
    return set_error(ANTS_E_ARG, "dims = %d must be 2 or 3", cfg->dims);
  if (cfg->dims == 3 && L.kind != ANTS_LRF_RZ && L.kind != ANTS_LRF_SLICED)
    return set_error(ANTS_E_ARG, "a 3-D search needs an r-z or sliced LRF");
  if (cfg->stat != ANTS_STAT_ML && cfg->stat != ANTS_STAT_CHI2)
    return set_error(ANTS_E_ARG, "unknown statistic %d", cfg->stat);
  if (cfg->start < ANTS_START_COG || cfg->start > ANTS_START_SEED)
    return set_error(ANTS_E_ARG, "unknown start option %d", cfg->start);
  if (cfg->start == ANTS_START_SEED && !d_seeds && n_events > 0)
    return set_error(ANTS_E_ARG, "start = SEED needs d_seeds");
  for (int a = 0; a < cfg->dims; ++a)
    if (!(cfg->step0[a] > 0.0 && isfinite(cfg->step0[a])))
      return set_error(ANTS_E_ARG, "step0[%d] = %g must be positive", a, cfg->step0[a]);
  if (!(cfg->h > 0.0 && isfinite(cfg->h)))
    return set_error(ANTS_E_ARG, "h = %g must be positive", cfg->h);
  if (!(cfg->edm_tol > 0.0 && isfinite(cfg->edm_tol)))
    return set_error(ANTS_E_ARG, "edm_tol = %g must be positive", cfg->edm_tol);
  if (cfg->max_iter < 0 || cfg->max_iter > 100000)
    return set_error(ANTS_E_ARG, "max_iter = %d outside 0..100000", cfg->max_iter);
  if (!(cfg->l_floor > 0.0) || !(cfg->v_floor > 0.0))
    return set_error(ANTS_E_ARG, "l_floor and v_floor must be positive");
  if (!isfinite(cfg->z_start)) return set_error(ANTS_E_ARG, "z_start not finite");
  if (n_events == 0) return ANTS_OK;
  if (!d_signals || !out.x || !out.y || !out.z || !out.E || !out.lnl || !out.chi2 || !out.ndf ||
      !out.status)
    return set_error(ANTS_E_ARG, "NULL signal or output pointer");
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != set->device) return set_error(ANTS_E_ARG, "LRF set lives on another device");
  SxP P;
  P = SxP{};
  P.L = L;
  P.dims = cfg->dims;
  P.stat = cfg->stat;
  P.start = cfg->start;
  P.max_iter = cfg->max_iter;
  for (int a = 0; a < 3; ++a) P.s0[a] = a < cfg->dims ? cfg->step0[a] : 0.0;
  P.z_start = cfg->z_start;
  P.h = cfg->h;
  P.edm = cfg->edm_tol;
  P.lfloor = cfg->l_floor;
  P.vfloor = cfg->v_floor;
  P.io.sig = d_signals;
  P.io.ld = set->ns;
  P.io.seeds = cfg->start == ANTS_START_SEED ? d_seeds : nullptr;
  P.io.x = out.x;
  P.io.y = out.y;
  P.io.z = out.z;
  P.io.E = out.E;
  P.io.lnl = out.lnl;
  P.io.chi2 = out.chi2;
  P.io.ndf = out.ndf;
  P.io.status = out.status;
  P.io.nfp = out.n_fp64;
  P.io.n = n_events;
  P.iters = d_iters;
  int64_t blocks = (n_events + 3) / 4;
  const int64_t cap = (int64_t)num_cu() * 16;
  if (blocks > cap) blocks = cap;
  hipError_t e = launch_search<true>(P, (int)blocks, (hipStream_t)hip_stream);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_reconstruct_migrad launch");
}
