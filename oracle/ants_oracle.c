/*
 * FP64 CPU oracle for contracting-grid event reconstruction (ANTS2,
 * arXiv:1602.07247).  TEST INFRASTRUCTURE ONLY: the library under
 * paper_1602_07247_amd/ never links, loads or calls this file.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark use it.
 *
 * Everything is plain double precision, one event at a time, written to be
 * checked against the paper by eye rather than to be fast.  Events are
 * independent, so an OpenMP loop over events gives the same bits as a
 * single thread.
 *
 * Passages followed:
 *   - centroid start position ........... Sec. 5.1.1, the CoG equation
 *   - start options (CoG / strongest) ... Sec. 5.1.2.1
 *   - statistic (ML or least squares) ... Sec. 5.1.2
 *   - contracting grid, energy ratio .... Sec. 5.1.2.2
 *   - passive sensors ................... Sec. 5.3
 *   - LRF as cubic B-splines (1-D axial, 2-D XY, r-z) ... Sec. 6, 6.1.1, 6.1.2
 *   - one LRF shared by a group with per-sensor relative gains ... Sec. 6.2
 *   - learned seed (fully connected ReLU net, trained by back-propagation)
 *     ... Sec. 5.1.3
 * Readings where the paper is silent are listed in the design notes; each
 * is restated where it is used below.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* status bits (same meaning as the library's; values restated here) */
#define O_EMPTY 1
#define O_BAD_INPUT 2
#define O_NO_ACTIVE 4
#define O_NO_VALID_NODE 8
#define O_FALLBACK 16
#define O_TIE 32

#define O_AXIAL 1
#define O_XY 2
#define O_RZ 3
#define O_COMPOSITE 4
#define O_SLICED 5

typedef struct {
  int kind;             /* 1 axial (r), 2 XY (x,y), 3 r-z (r,z)          */
  int n_sensors;
  const double* sxy;    /* [n][2] sensor centres (mm)                     */
  const double* gain;   /* [n] relative gain                              */
  const uint8_t* active;/* [n] 0 = passive                                */
  int shared;           /* 1: one coefficient table for all sensors       */
  int nb[2];            /* breakpoints per axis, both ends included       */
  double lo[2], hi[2];  /* spline domain per axis                         */
  const double* coef;   /* [n_lrf][nb[1]+2][nb[0]+2] (axis 1 unused = 1 row);
                           sliced: [n_lrf][n_planes][nb[1]+2][nb[0]+2]     */
  /* composite (kind 4, Sec. 6.1.1): the fields above hold the axial part
   * (one table shared by all sensors), these the XY residual added to it */
  int xy_nb[2];
  double xy_lo[2], xy_hi[2];
  const double* xy_coef;  /* [n_xy][xy_nb[1]+2][xy_nb[0]+2]                 */
  int xy_shared;
  /* sliced (kind 5, Sec. 6.1.2): XY LRFs on n_planes z planes at
   * z_lo + p (z_hi - z_lo) / (n_planes - 1)                                */
  int n_planes;
  double z_lo, z_hi;
} o_lrf;

typedef struct {
  int nodes[3];
  int iterations;
  double shrink;
  double step0[3];
  double z_start;
  int stat;             /* 0 ML, 1 chi2 */
  int start;            /* 0 CoG, 1 strongest sensor, 2 seed */
  double l_floor, v_floor;
  /* seed refinement: per-event steps from the seed's log-variance */
  int seed_steps;
  double seed_kappa;
  int seed_kmin, seed_kmax;
  double seed_scale[3];
  /* sensor cuts (Sec. 5.1.2): ignore sensors with a signal below
   * cut_signal, or farther (in x-y) than cut_distance from the start
   * position; <= 0 disables a cut */
  double cut_signal, cut_distance;
} o_cfg;

/* ------------------------------------------------------------------ */
/* Cubic B-spline on a uniform extended knot vector (Sec. 6, reading:   */
/* breakpoints lo + m*d, m = 0..nb-1, and nb+2 coefficients; coefficient */
/* j belongs to the B-spline centred on breakpoint j-1).                 */
/* ------------------------------------------------------------------ */

/* Uniform cubic B-spline basis on one interval, t in [0,1]. */
void o_basis(double t, double b[4]) {
  double s = 1.0 - t;
  b[0] = s * s * s / 6.0;
  b[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
  b[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
  b[3] = t * t * t / 6.0;
}

/* Derivative of the basis with respect to t. */
static void o_basis_dt(double t, double b[4]) {
  double s = 1.0 - t;
  b[0] = -0.5 * s * s;
  b[1] = (9.0 * t * t - 12.0 * t) / 6.0;
  b[2] = (-9.0 * t * t + 6.0 * t + 3.0) / 6.0;
  b[3] = 0.5 * t * t;
}

/* Locate u: returns 0 when u is outside [lo,hi] (with a relative slack of
 * 1e-9 of the span, so grid nodes placed on a domain edge by floating-point
 * arithmetic stay inside); else the interval m and local coordinate t. */
static int o_locate(double u, int nb, double lo, double hi, int* m, double* t) {
  double span = hi - lo;
  double tol = 1e-9 * span;
  if (!(u >= lo - tol && u <= hi + tol)) return 0;
  int nint = nb - 1;
  double d = span / nint;
  double v = (u - lo) / d;
  int k = (int)floor(v);
  if (k < 0) k = 0;
  if (k > nint - 1) k = nint - 1;
  *m = k;
  *t = v - k;
  return 1;
}

/* 1-D spline value; 0 outside the domain. */
double o_spline1(const double* c, int nb, double lo, double hi, double u) {
  int m;
  double t, b[4];
  if (!o_locate(u, nb, lo, hi, &m, &t)) return 0.0;
  o_basis(t, b);
  return c[m] * b[0] + c[m + 1] * b[1] + c[m + 2] * b[2] + c[m + 3] * b[3];
}

/* 1-D spline derivative d/du; 0 outside the domain. */
double o_spline1_du(const double* c, int nb, double lo, double hi, double u) {
  int m;
  double t, b[4];
  if (!o_locate(u, nb, lo, hi, &m, &t)) return 0.0;
  o_basis_dt(t, b);
  double d = (hi - lo) / (nb - 1);
  return (c[m] * b[0] + c[m + 1] * b[1] + c[m + 2] * b[2] + c[m + 3] * b[3]) / d;
}

/* 2-D tensor-product spline, coefficient table [nb1+2][nb0+2]; u on axis 0. */
double o_spline2(const double* c, const int nb[2], const double lo[2], const double hi[2],
                 double u, double w, double* du, double* dw) {
  int m0, m1;
  double t0, t1, b0[4], b1[4], d0[4], d1[4];
  if (du) *du = 0.0;
  if (dw) *dw = 0.0;
  if (!o_locate(u, nb[0], lo[0], hi[0], &m0, &t0)) return 0.0;
  if (!o_locate(w, nb[1], lo[1], hi[1], &m1, &t1)) return 0.0;
  o_basis(t0, b0);
  o_basis(t1, b1);
  o_basis_dt(t0, d0);
  o_basis_dt(t1, d1);
  int ld = nb[0] + 2;
  double v = 0.0, vu = 0.0, vw = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int q = 0; q < 4; ++q) {
      double cc = c[(m1 + a) * ld + (m0 + q)];
      v += cc * b1[a] * b0[q];
      vu += cc * b1[a] * d0[q];
      vw += cc * d1[a] * b0[q];
    }
  if (du) *du = vu / ((hi[0] - lo[0]) / (nb[0] - 1));
  if (dw) *dw = vw / ((hi[1] - lo[1]) / (nb[1] - 1));
  return v;
}

/* Independent evaluator for the pins: Cox-de Boor recursion on the full
 * extended knot vector knots[k] = lo + (k-3)*d, k = 0..nc+3.  Shares no
 * arithmetic with o_basis. */
double o_deboor1(const double* c, int nb, double lo, double hi, double u) {
  int nc = nb + 2;
  double d = (hi - lo) / (nb - 1);
  int nk = nc + 4;
  double knots[512];
  if (nk > 512) return NAN;
  for (int k = 0; k < nk; ++k) knots[k] = lo + (k - 3) * d;
  if (u < lo || u > hi) return 0.0;
  /* span index mu with knots[mu] <= u < knots[mu+1], restricted to the
   * domain spans 3 .. nc-1 */
  int mu = 3;
  while (mu < nc - 1 && u >= knots[mu + 1]) ++mu;
  /* degree-0 .. degree-3 basis via the recursion */
  double N[4][4];
  memset(N, 0, sizeof(N));
  N[0][0] = 1.0; /* B_{mu,0} */
  for (int p = 1; p <= 3; ++p) {
    /* N[p][r] holds B_{mu-p+r, p} for r = 0..p */
    for (int r = 0; r <= p; ++r) {
      int j = mu - p + r;
      double left = 0.0, right = 0.0;
      if (r - 1 >= 0) {
        double den = knots[j + p] - knots[j];
        left = (u - knots[j]) / den * N[p - 1][r - 1];
      }
      if (r <= p - 1) {
        double den = knots[j + p + 1] - knots[j + 1];
        right = (knots[j + p + 1] - u) / den * N[p - 1][r];
      }
      N[p][r] = left + right;
    }
  }
  double v = 0.0;
  for (int r = 0; r <= 3; ++r) v += c[mu - 3 + r] * N[3][r];
  return v;
}

/* ------------------------------------------------------------------ */
/* LRF of sensor i at a source position (Sec. 6): max(spline, 0) inside */
/* the domain, 0 outside (reading).                                     */
/* ------------------------------------------------------------------ */
static const double* o_table(const o_lrf* L, int i) {
  size_t per = (size_t)(L->nb[0] + 2) *
               (size_t)((L->kind == O_AXIAL || L->kind == O_COMPOSITE) ? 1 : (L->nb[1] + 2));
  if (L->kind == O_SLICED) per *= (size_t)L->n_planes;
  return L->coef + (L->shared ? 0 : (size_t)i * per);
}

double o_lrf_value(const o_lrf* L, int i, double x, double y, double z) {
  double dx = x - L->sxy[2 * i], dy = y - L->sxy[2 * i + 1];
  double v;
  if (L->kind == O_AXIAL) {
    double r = sqrt(dx * dx + dy * dy);
    v = o_spline1(o_table(L, i), L->nb[0], L->lo[0], L->hi[0], r);
  } else if (L->kind == O_XY) {
    v = o_spline2(o_table(L, i), L->nb, L->lo, L->hi, x, y, NULL, NULL);
  } else if (L->kind == O_COMPOSITE) {
    /* Sec. 6.1.1: the sum of an axial LRF and an XY LRF (the residual);
     * reading: each part is 0 outside its own domain, the sum is clamped */
    double r = sqrt(dx * dx + dy * dy);
    double a = o_spline1(L->coef, L->nb[0], L->lo[0], L->hi[0], r);
    size_t per = (size_t)(L->xy_nb[0] + 2) * (size_t)(L->xy_nb[1] + 2);
    const double* t = L->xy_coef + (L->xy_shared ? 0 : (size_t)i * per);
    v = a + o_spline2(t, L->xy_nb, L->xy_lo, L->xy_hi, x, y, NULL, NULL);
  } else if (L->kind == O_SLICED) {
    /* Sec. 6.1.2: XY LRFs on z planes, linear interpolation in z between
     * the values of the two closest planes; reading: 0 outside the planes'
     * z range (with the domain slack) */
    int p;
    double t;
    if (!o_locate(z, L->n_planes, L->z_lo, L->z_hi, &p, &t)) return 0.0;
    const double* c = o_table(L, i);
    size_t plane = (size_t)(L->nb[0] + 2) * (size_t)(L->nb[1] + 2);
    double a = o_spline2(c + (size_t)p * plane, L->nb, L->lo, L->hi, x, y, NULL, NULL);
    double b = o_spline2(c + (size_t)(p + 1) * plane, L->nb, L->lo, L->hi, x, y, NULL, NULL);
    a = a > 0.0 ? a : 0.0;
    b = b > 0.0 ? b : 0.0;
    return (1.0 - t) * a + t * b;
  } else {
    double r = sqrt(dx * dx + dy * dy);
    v = o_spline2(o_table(L, i), L->nb, L->lo, L->hi, r, z, NULL, NULL);
  }
  return v > 0.0 ? v : 0.0;
}

/* Gradient of the LRF with respect to (x, y, z); zero where the LRF is
 * clamped to 0.  Used by the Cramer-Rao bound only. */
static double o_lrf_grad(const o_lrf* L, int i, double x, double y, double z, double g[3]) {
  double dx = x - L->sxy[2 * i], dy = y - L->sxy[2 * i + 1];
  double v = 0.0;
  g[0] = g[1] = g[2] = 0.0;
  if (L->kind == O_AXIAL) {
    double r = sqrt(dx * dx + dy * dy);
    const double* c = o_table(L, i);
    v = o_spline1(c, L->nb[0], L->lo[0], L->hi[0], r);
    double dr = o_spline1_du(c, L->nb[0], L->lo[0], L->hi[0], r);
    if (r > 0) { g[0] = dr * dx / r; g[1] = dr * dy / r; }
  } else if (L->kind == O_XY) {
    double du, dw;
    v = o_spline2(o_table(L, i), L->nb, L->lo, L->hi, x, y, &du, &dw);
    g[0] = du; g[1] = dw;
  } else {
    double r = sqrt(dx * dx + dy * dy), du, dw;
    v = o_spline2(o_table(L, i), L->nb, L->lo, L->hi, r, z, &du, &dw);
    if (r > 0) { g[0] = du * dx / r; g[1] = du * dy / r; }
    g[2] = dw;
  }
  if (v <= 0.0) { g[0] = g[1] = g[2] = 0.0; return 0.0; }
  return v;
}

/* ------------------------------------------------------------------ */
/* Match statistic at one node (Sec. 5.1.2 and 5.1.2.2).                */
/*   S  = sum over active sensors of g_i L_i                            */
/*   A  = N / S          (the energy ratio of Sec. 5.1.2.2)             */
/*   mu_i = A g_i L_i                                                   */
/*   ML: l = sum [ n_i ln(A g_i max(L_i, l_floor)) - mu_i ] with the    */
/*       n_i = 0 terms reduced to -mu_i (0 ln 0 = 0); the constant      */
/*       -sum ln n_i! is dropped (reading).  Minimised quantity: -l.    */
/*   chi2 = sum (n_i - mu_i)^2 / max(mu_i, v_floor)                     */
/* Returns the minimised statistic, +inf when S <= 0 or not finite.     */
/* ------------------------------------------------------------------ */
typedef struct { double stat, S, A, lnl, chi2; } o_node;

o_node o_node_eval(const o_lrf* L, const o_cfg* C, const double* n, double N,
                   double x, double y, double z) {
  o_node r;
  double S = 0.0;
  int ns = L->n_sensors;
  double* Lv = (double*)malloc(sizeof(double) * (size_t)ns);
  for (int i = 0; i < ns; ++i) {
    if (!L->active[i]) { Lv[i] = 0.0; continue; }
    Lv[i] = o_lrf_value(L, i, x, y, z);
    S += L->gain[i] * Lv[i];
  }
  r.S = S;
  if (!(S > 0.0) || !isfinite(S)) {
    r.stat = INFINITY; r.A = NAN; r.lnl = NAN; r.chi2 = NAN;
    free(Lv);
    return r;
  }
  double A = N / S;
  double lnl = 0.0, chi2 = 0.0;
  for (int i = 0; i < ns; ++i) {
    if (!L->active[i]) continue;
    double mu = A * L->gain[i] * Lv[i];
    double Lt = Lv[i] > C->l_floor ? Lv[i] : C->l_floor;
    if (n[i] > 0.0) lnl += n[i] * log(A * L->gain[i] * Lt);
    lnl -= mu;
    double var = mu > C->v_floor ? mu : C->v_floor;
    chi2 += (n[i] - mu) * (n[i] - mu) / var;
  }
  free(Lv);
  r.A = A; r.lnl = lnl; r.chi2 = chi2;
  r.stat = (C->stat == 0) ? -lnl : chi2;
  if (!isfinite(r.stat)) r.stat = INFINITY;
  return r;
}

/* Tie tolerance (reading; the paper is silent on ties).  Two node
 * statistics count as equal when they differ by at most O_TIE_REL times the
 * event's summed signal N (for either statistic).  That is far above the
 * rounding of a double-precision evaluation, which depends on the order of
 * the sums and on the logarithm's implementation, and far below the gaps
 * that separate distinct nodes, so mathematically equal nodes are ordered by
 * index and every other decision is unchanged. */
#define O_TIE_REL 1e-12

/* Node coordinates on the grid of one iteration (Sec. 5.1.2.2: a regular
 * grid centred at the current centre).  Node index (jz*ny + jy)*nx + jx. */
static void o_node_pos(const o_cfg* C, const double c[3], const double s[3], int j, double p[3]) {
  int nx = C->nodes[0], ny = C->nodes[1];
  int jx = j % nx, jy = (j / nx) % ny, jz = j / (nx * ny);
  p[0] = c[0] + (double)(jx - (nx - 1) / 2) * s[0];
  p[1] = c[1] + (double)(jy - (ny - 1) / 2) * s[1];
  p[2] = c[2] + (double)(jz - (C->nodes[2] - 1) / 2) * s[2];
}

/* ------------------------------------------------------------------ */
/* One event.  Outputs: x,y,z,E,lnl,chi2,ndf,status and per-iteration  */
/* best node index and gap between the two best statistics.            */
/* ------------------------------------------------------------------ */
void o_event(const o_lrf* L, const o_cfg* C, const double* n, const double* seed,
             double out[6], int* ndf, int* status, int* path, double* gaps) {
  int ns = L->n_sensors;
  int na = 0, bad = 0;
  double N = 0.0;
  *status = 0;
  for (int i = 0; i < ns; ++i) {
    if (!L->active[i]) continue;
    ++na;
    if (!isfinite(n[i]) || n[i] < 0.0) bad = 1;
    else N += n[i];
  }
  int dim = (C->nodes[2] > 1) ? 3 : 2;
  *ndf = na - (dim + 1);
  for (int k = 0; k < 6; ++k) out[k] = NAN;
  for (int k = 0; k < C->iterations; ++k) { if (path) path[k] = -1; if (gaps) gaps[k] = NAN; }
  if (na == 0) { *status = O_NO_ACTIVE; return; }
  if (bad) { *status = O_BAD_INPUT; return; }
  if (!(N > 0.0)) { *status = O_EMPTY; return; }

  /* start position (Sec. 5.1.1 centroid, or Sec. 5.1.2.1 strongest sensor) */
  double c[3];
  if (C->start == 2 && seed) {
    c[0] = seed[0]; c[1] = seed[1]; c[2] = seed[2];
  } else if (C->start == 1) {
    int best = -1;
    for (int i = 0; i < ns; ++i)
      if (L->active[i] && (best < 0 || n[i] > n[best])) best = i;
    c[0] = L->sxy[2 * best]; c[1] = L->sxy[2 * best + 1]; c[2] = C->z_start;
  } else {
    double sw = 0.0, sx = 0.0, sy = 0.0;
    for (int i = 0; i < ns; ++i) {
      if (!L->active[i]) continue;
      double w = n[i] / L->gain[i];
      sw += w; sx += L->sxy[2 * i] * w; sy += L->sxy[2 * i + 1] * w;
    }
    c[0] = sx / sw; c[1] = sy / sw; c[2] = C->z_start;
  }
  if (dim == 2) c[2] = C->z_start;

  /* Sensor cuts (Sec. 5.1.2).  Reading: the start position uses every
   * active sensor; the ignored ones then leave the statistic, the energy
   * ratio, the outputs and ndf for the whole event, exactly as if they were
   * passive. */
  uint8_t* use = NULL;
  o_lrf Lcut;
  if (C->cut_signal > 0.0 || C->cut_distance > 0.0) {
    use = (uint8_t*)malloc((size_t)ns);
    int nu = 0;
    N = 0.0;
    for (int i = 0; i < ns; ++i) {
      int u = L->active[i] != 0;
      if (u && C->cut_signal > 0.0 && n[i] < C->cut_signal) u = 0;
      if (u && C->cut_distance > 0.0) {
        double dx = L->sxy[2 * i] - c[0], dy = L->sxy[2 * i + 1] - c[1];
        if (sqrt(dx * dx + dy * dy) > C->cut_distance) u = 0;
      }
      use[i] = (uint8_t)u;
      if (u) { ++nu; N += n[i]; }
    }
    Lcut = *L;
    Lcut.active = use;
    L = &Lcut;
    *ndf = nu - (dim + 1);
    if (nu == 0) { *status = O_NO_ACTIVE; free(use); return; }
    if (!(N > 0.0)) { *status = O_EMPTY; free(use); return; }
  }

  int nn = C->nodes[0] * C->nodes[1] * C->nodes[2];
  double s[3] = {C->step0[0], C->step0[1], C->step0[2]};
  int K = C->iterations;
  if (C->start == 2 && seed && C->seed_steps) {
    /* Refinement of a seed (x, y, z, log-variance): the grid ends on the
     * configured final step s_f = step0 * shrink^(K-1); the event runs the
     * smallest number of iterations in [kmin, kmax] whose first step
     * s_f / shrink^(k-1) reaches kappa * sigma on every searched axis, with
     * sigma = seed_scale * exp(log-variance / 2). */
    double sf[3];
    for (int a = 0; a < 3; ++a) {
      sf[a] = C->step0[a];
      for (int k = 1; k < C->iterations; ++k) sf[a] *= C->shrink;
    }
    double need = exp(0.5 * seed[3]) * C->seed_kappa;
    int k = 0;
    for (; k < C->seed_kmin - 1; ++k)
      for (int a = 0; a < 3; ++a) sf[a] = sf[a] / C->shrink;
    if (!isfinite(need)) {
      for (; k < C->seed_kmax - 1; ++k)
        for (int a = 0; a < 3; ++a) sf[a] = sf[a] / C->shrink;
    } else {
      for (;;) {
        int short_ = 0;
        for (int a = 0; a < 3; ++a)
          if (C->nodes[a] > 1 && sf[a] < need * C->seed_scale[a]) short_ = 1;
        if (!short_ || k >= C->seed_kmax - 1) break;
        for (int a = 0; a < 3; ++a) sf[a] = sf[a] / C->shrink;
        ++k;
      }
    }
    K = k + 1;
    for (int a = 0; a < 3; ++a) s[a] = sf[a];
  }
  double* st = (double*)malloc(sizeof(double) * (size_t)nn);
  for (int k = 0; k < K; ++k) {
    double b1 = INFINITY, b2 = INFINITY;
    for (int j = 0; j < nn; ++j) {
      double p[3];
      o_node_pos(C, c, s, j, p);
      st[j] = o_node_eval(L, C, n, N, p[0], p[1], p[2]).stat;
      if (st[j] < b1) { b2 = b1; b1 = st[j]; }
      else if (st[j] < b2) { b2 = st[j]; }
    }
    /* The best node: the lowest index among the nodes whose statistic is
     * within the tie tolerance of the minimum (reading: the paper does not
     * order equally good nodes; values that differ only by rounding are
     * equal, and equal nodes go to the lowest index, x fastest). */
    int j1 = -1, nties = 0;
    if (b1 < INFINITY) {
      double tol = O_TIE_REL * N;
      for (int j = 0; j < nn; ++j)
        if (st[j] <= b1 + tol) {
          if (j1 < 0) j1 = j;
          ++nties;
        }
    }
    if (path) path[k] = j1;
    if (gaps) gaps[k] = b2 - b1;
    if (j1 < 0) {            /* every node invalid: keep the centre */
      *status |= O_NO_VALID_NODE;
    } else {
      if (nties > 1) *status |= O_TIE;   /* a tie, resolved by index */
      double p[3];
      o_node_pos(C, c, s, j1, p);
      c[0] = p[0]; c[1] = p[1]; c[2] = p[2];
    }
    s[0] *= C->shrink; s[1] *= C->shrink; s[2] *= C->shrink;
  }
  free(st);
  o_node r = o_node_eval(L, C, n, N, c[0], c[1], c[2]);
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2];
  out[3] = r.A; out[4] = r.lnl; out[5] = r.chi2;
  free(use);
}

/* Batch over events; signals [n_ev][n_sensors] as double. */
void o_reconstruct(const o_lrf* L, const o_cfg* C, int64_t n_ev, const double* sig,
                   const double* seeds, double* out6, int* ndf, int* status,
                   int* path, double* gaps, int n_threads) {
  int K = C->iterations;
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
  for (int64_t e = 0; e < n_ev; ++e) {
    o_event(L, C, sig + e * L->n_sensors, seeds ? seeds + 4 * e : NULL, out6 + 6 * e,
            ndf + e, status + e, path ? path + e * K : NULL, gaps ? gaps + e * K : NULL);
  }
}

/* Statistic of every node of an arbitrary lattice (for brute-force pins). */
void o_lattice_stats(const o_lrf* L, const o_cfg* C, const double* n, const double c[3],
                     const double s[3], const int nodes[3], double* stats, int n_threads) {
  double N = 0.0;
  for (int i = 0; i < L->n_sensors; ++i) if (L->active[i]) N += n[i];
  int64_t nn = (int64_t)nodes[0] * nodes[1] * nodes[2];
#pragma omp parallel for schedule(static) num_threads(n_threads)
  for (int64_t j = 0; j < nn; ++j) {
    int64_t jx = j % nodes[0], jy = (j / nodes[0]) % nodes[1], jz = j / ((int64_t)nodes[0] * nodes[1]);
    double x = c[0] + (double)(jx - (nodes[0] - 1) / 2) * s[0];
    double y = c[1] + (double)(jy - (nodes[1] - 1) / 2) * s[1];
    double z = c[2] + (double)(jz - (nodes[2] - 1) / 2) * s[2];
    stats[j] = o_node_eval(L, C, n, N, x, y, z).stat;
  }
}

/* Node evaluation exposed for pins: returns stat and fills S, A, lnl, chi2. */
void o_node_eval_ext(const o_lrf* L, const o_cfg* C, const double* n, double x, double y,
                     double z, double res[5]) {
  double N = 0.0;
  for (int i = 0; i < L->n_sensors; ++i) if (L->active[i]) N += n[i];
  o_node r = o_node_eval(L, C, n, N, x, y, z);
  res[0] = r.stat; res[1] = r.S; res[2] = r.A; res[3] = r.lnl; res[4] = r.chi2;
}

/* LRF values for many positions: vals[p][i]. */
void o_lrf_values(const o_lrf* L, int64_t n_pos, const double* pos3, double* vals, int n_threads) {
#pragma omp parallel for schedule(static) num_threads(n_threads)
  for (int64_t p = 0; p < n_pos; ++p)
    for (int i = 0; i < L->n_sensors; ++i)
      vals[p * L->n_sensors + i] = o_lrf_value(L, i, pos3[3 * p], pos3[3 * p + 1], pos3[3 * p + 2]);
}

/* Expected counts for event generation: mu_i = A g_i L_i with
 * A = E_tot / sum_active g_i L_i (the total expected photoelectrons over
 * active sensors equals E_tot).  Passive sensors get 0. */
void o_expected_counts(const o_lrf* L, int64_t n_pos, const double* pos3, const double* etot,
                       double* mu, int n_threads) {
#pragma omp parallel for schedule(static) num_threads(n_threads)
  for (int64_t p = 0; p < n_pos; ++p) {
    double S = 0.0;
    double* m = mu + p * L->n_sensors;
    for (int i = 0; i < L->n_sensors; ++i) {
      m[i] = L->active[i] ? L->gain[i] * o_lrf_value(L, i, pos3[3 * p], pos3[3 * p + 1], pos3[3 * p + 2]) : 0.0;
      S += m[i];
    }
    double A = S > 0 ? etot[p] / S : 0.0;
    for (int i = 0; i < L->n_sensors; ++i) m[i] *= A;
  }
}

/* Cramer-Rao bound on (x, y[, z]) at the true position for Poisson counts
 * with means mu_i = A g_i L_i(x,y,z); parameters theta = (x, y, [z], A).
 * Fisher information I_jk = sum_i d_j mu_i d_k mu_i / mu_i.
 * Writes the diagonal of I^-1 for the position parameters. */
void o_crb(const o_lrf* L, int dim, int64_t n_pos, const double* pos3, const double* A,
           double* var_out /* [n][dim] */) {
  for (int64_t p = 0; p < n_pos; ++p) {
    int np = dim + 1;
    double I[4][4];
    memset(I, 0, sizeof(I));
    for (int i = 0; i < L->n_sensors; ++i) {
      if (!L->active[i]) continue;
      double g[3];
      double v = o_lrf_grad(L, i, pos3[3 * p], pos3[3 * p + 1], pos3[3 * p + 2], g);
      double mu = A[p] * L->gain[i] * v;
      if (!(mu > 0)) continue;
      double d[4];
      for (int a = 0; a < dim; ++a) d[a] = A[p] * L->gain[i] * g[a];
      d[dim] = L->gain[i] * v;
      for (int a = 0; a < np; ++a)
        for (int b = 0; b < np; ++b) I[a][b] += d[a] * d[b] / mu;
    }
    /* invert the small symmetric matrix by Gauss-Jordan */
    double M[4][8];
    for (int a = 0; a < np; ++a)
      for (int b = 0; b < 2 * np; ++b) M[a][b] = (b < np) ? I[a][b] : (b - np == a ? 1.0 : 0.0);
    int ok = 1;
    for (int col = 0; col < np; ++col) {
      int piv = col;
      for (int r = col + 1; r < np; ++r) if (fabs(M[r][col]) > fabs(M[piv][col])) piv = r;
      if (M[piv][col] == 0.0) { ok = 0; break; }
      if (piv != col) for (int b = 0; b < 2 * np; ++b) { double t = M[col][b]; M[col][b] = M[piv][b]; M[piv][b] = t; }
      double inv = 1.0 / M[col][col];
      for (int b = 0; b < 2 * np; ++b) M[col][b] *= inv;
      for (int r = 0; r < np; ++r) {
        if (r == col) continue;
        double f = M[r][col];
        for (int b = 0; b < 2 * np; ++b) M[r][b] -= f * M[col][b];
      }
    }
    for (int a = 0; a < dim; ++a) var_out[p * dim + a] = ok ? M[a][np + a] : NAN;
  }
}

/* ------------------------------------------------------------------ */
/* Reference for the flood-field generator (Sec. 4.1.1 flood field):     */
/* Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw (SC'11),  */
/* and Poisson draws by sequential-search inversion (mean < 10) or the   */
/* transformed rejection method with squeeze of Hoermann (1993).         */
/* ------------------------------------------------------------------ */
void o_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t n[4];
    n[0] = (uint32_t)(p1 >> 32) ^ c[1] ^ k[0];
    n[1] = (uint32_t)p1;
    n[2] = (uint32_t)(p0 >> 32) ^ c[3] ^ k[1];
    n[3] = (uint32_t)p0;
    memcpy(c, n, sizeof(c));
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
  memcpy(out, c, sizeof(c));
}

static double o_u53(uint32_t a, uint32_t b) {
  uint64_t bits = (((uint64_t)a << 32) | b) >> 11;
  return ((double)bits + 0.5) / 9007199254740992.0; /* 2^53 */
}

static void o_draw(uint64_t ev, uint32_t stream, uint32_t call, const uint32_t key[2], uint32_t w[4]) {
  uint32_t ctr[4] = {(uint32_t)ev, (uint32_t)(ev >> 32), stream, call};
  o_philox4x32_10(ctr, key, w);
}

double o_poisson(double mu, uint64_t ev, uint32_t stream, const uint32_t key[2]) {
  uint32_t w[4];
  if (!(mu > 0.0)) return 0.0;
  if (mu < 10.0) {
    o_draw(ev, stream, 0, key, w);
    double u = o_u53(w[0], w[1]);
    double p = exp(-mu), cdf = p;
    int k = 0;
    while (u > cdf && k < 1000) { ++k; p = p * (mu / k); cdf += p; }
    return (double)k;
  }
  double sq = sqrt(mu), lmu = log(mu);
  double b = 0.931 + 2.53 * sq;
  double a = -0.059 + 0.02483 * b;
  double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
  double v_r = 0.9277 - 3.6224 / (b - 2.0);
  for (uint32_t t = 0; t < 64; ++t) {
    o_draw(ev, stream, t, key, w);
    double U = o_u53(w[0], w[1]) - 0.5;
    double V = o_u53(w[2], w[3]);
    double us = 0.5 - fabs(U);
    double k = floor((2.0 * a / us + b) * U + mu + 0.43);
    if (us >= 0.07 && V <= v_r) return k;
    if (k < 0.0 || (us < 0.013 && V > us)) continue;
    if (log(V) + log(inv_alpha) - log(a / (us * us) + b) <= -mu + k * lmu - lgamma(k + 1.0)) return k;
  }
  return floor(mu + 0.5);
}

/* Events first..first+n-1: truth4 [n][4] = (x, y, z, E_tot), signals [n][ns]. */
void o_generate(const o_lrf* L, int region, double extent, double z_lo, double z_hi, double e_lo,
                double e_hi, int noiseless, uint64_t seed, uint64_t first, int64_t n,
                double* truth4, double* sig, int n_threads) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static) num_threads(n_threads)
  for (int64_t e = 0; e < n; ++e) {
    uint64_t ev = first + (uint64_t)e;
    uint32_t wa[4], wb[4];
    o_draw(ev, 0xFFFFFFFFu, 0, key, wa);
    o_draw(ev, 0xFFFFFFFFu, 1, key, wb);
    double u1 = o_u53(wa[0], wa[1]), u2 = o_u53(wa[2], wa[3]);
    double u3 = o_u53(wb[0], wb[1]), u4 = o_u53(wb[2], wb[3]);
    double x, y;
    if (region == 0) {
      double r = extent * sqrt(u1), phi = 2.0 * M_PI * u2;
      x = r * cos(phi); y = r * sin(phi);
    } else {
      x = -extent + 2.0 * extent * u1; y = -extent + 2.0 * extent * u2;
    }
    double z = z_hi > z_lo ? z_lo + (z_hi - z_lo) * u3 : z_lo;
    double E = e_lo + (e_hi - e_lo) * u4;
    double* row = sig + e * L->n_sensors;
    double S = 0.0;
    for (int i = 0; i < L->n_sensors; ++i) {
      row[i] = L->active[i] ? L->gain[i] * o_lrf_value(L, i, x, y, z) : 0.0;
      S += row[i];
    }
    double A = S > 0.0 ? E / S : 0.0;
    for (int i = 0; i < L->n_sensors; ++i) {
      if (!L->active[i]) continue;
      double mu = A * row[i];
      row[i] = noiseless ? mu : o_poisson(mu, ev, (uint32_t)i, key);
    }
    truth4[4 * e] = x; truth4[4 * e + 1] = y; truth4[4 * e + 2] = z; truth4[4 * e + 3] = E;
  }
}

/* Seeded reconstruction: refine from the seed; events whose chi2/ndf at the
 * refined node exceeds chi2ndf_max (or is not finite, or ndf <= 0) are
 * reconstructed again with the fallback grid and flagged (status bit 16). */
void o_reconstruct_seeded(const o_lrf* L, const o_cfg* R, const o_cfg* F, double chi2ndf_max,
                          int64_t n_ev, const double* sig, const double* seeds, double* out6,
                          int* ndf, int* status, int n_threads) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
  for (int64_t e = 0; e < n_ev; ++e) {
    const double* row = sig + e * L->n_sensors;
    o_event(L, R, row, seeds + 4 * e, out6 + 6 * e, ndf + e, status + e, NULL, NULL);
    if (status[e] & (O_EMPTY | O_BAD_INPUT | O_NO_ACTIVE)) continue;
    double q = out6[6 * e + 5];
    if (ndf[e] > 0 && q / ndf[e] <= chi2ndf_max) continue;
    o_event(L, F, row, NULL, out6 + 6 * e, ndf + e, status + e, NULL, NULL);
    status[e] |= O_FALLBACK;
  }
}

/* ------------------------------------------------------------------ */
/* Simplex search (Sec. 5.1.2.1: the Minuit2 Simplex minimiser over x, y  */
/* or x, y, z from the centroid or the strongest sensor).  Minuit2 itself */
/* is not available; this is the Nelder-Mead method as defined by         */
/* Lagarias, Reeds, Wright and Wright (SIAM J. Optim. 9, 1998), with the  */
/* standard coefficients: reflection 1, expansion 2, contraction 1/2,     */
/* shrink 1/2.  Readings:                                                 */
/*  - the energy is not a free parameter: at every point it is the ratio  */
/*    of the sums (as for the grid), so the search is over position only; */
/*  - initial simplex: the start point and the start point moved by       */
/*    step0[a] along each searched axis a;                                 */
/*  - values within the tie tolerance (O_TIE_REL * N) are equal; vertices */
/*    are kept ordered by value, a new vertex going after the vertices    */
/*    whose value equals its own, and the best vertex staying first after */
/*    a shrink when tied;                                                  */
/*  - stop when every vertex lies within tol (mm) of the best one on      */
/*    every searched axis, or after max_iter iterations (an iteration is  */
/*    one reflection step with its expansion, contraction or shrink).     */
/* Arithmetic is written out step by step (no fused multiply-add).        */
/* ------------------------------------------------------------------ */
typedef struct {
  int dims;             /* 2: x, y;  3: x, y, z                          */
  int stat;             /* 0 ML, 1 chi2                                  */
  int start;            /* 0 CoG, 1 strongest sensor, 2 seed             */
  double step0[3];      /* initial simplex edge per axis (mm)            */
  double z_start;
  double tol;           /* convergence size (mm)                          */
  int max_iter;
  double l_floor, v_floor;
} o_scfg;

typedef struct { double p[3]; double f; } o_vtx;

static int o_lt(double a, double b, double tol) { return a < b - tol; }

/* insert w into v[0..n-1] (ordered) after every vertex whose value is not
 * above w's (within the tolerance): v becomes n+1 ordered vertices */
static void o_sx_insert(o_vtx* v, int n, o_vtx w, double tol) {
  int pos = n;
  while (pos > 0 && o_lt(w.f, v[pos - 1].f, tol)) { v[pos] = v[pos - 1]; --pos; }
  v[pos] = w;
}

void o_simplex_event(const o_lrf* L, const o_scfg* S, const double* n, const double* seed,
                     double out[6], int* ndf, int* status, int* iters, int* evals) {
  int ns = L->n_sensors, na = 0, bad = 0, d = S->dims;
  double N = 0.0;
  *status = 0;
  *iters = 0;
  *evals = 0;
  for (int i = 0; i < ns; ++i) {
    if (!L->active[i]) continue;
    ++na;
    if (!isfinite(n[i]) || n[i] < 0.0) bad = 1;
    else N += n[i];
  }
  *ndf = na - (d + 1);
  for (int k = 0; k < 6; ++k) out[k] = NAN;
  if (na == 0) { *status = O_NO_ACTIVE; return; }
  if (bad) { *status = O_BAD_INPUT; return; }
  if (!(N > 0.0)) { *status = O_EMPTY; return; }
  /* statistic settings shared with the grid's node evaluation */
  o_cfg C;
  memset(&C, 0, sizeof(C));
  C.stat = S->stat;
  C.l_floor = S->l_floor;
  C.v_floor = S->v_floor;
  /* start (Sec. 5.1.1 centroid, Sec. 5.1.2.1 strongest sensor, or seed) */
  double c0[3] = {0.0, 0.0, S->z_start};
  if (S->start == 2 && seed) {
    c0[0] = seed[0]; c0[1] = seed[1];
    if (d == 3) c0[2] = seed[2];
  } else if (S->start == 1) {
    int best = -1;
    for (int i = 0; i < ns; ++i)
      if (L->active[i] && (best < 0 || n[i] > n[best])) best = i;
    c0[0] = L->sxy[2 * best]; c0[1] = L->sxy[2 * best + 1];
  } else {
    double sw = 0.0, sx = 0.0, sy = 0.0;
    for (int i = 0; i < ns; ++i) {
      if (!L->active[i]) continue;
      double w = n[i] / L->gain[i];
      sw += w; sx += L->sxy[2 * i] * w; sy += L->sxy[2 * i + 1] * w;
    }
    c0[0] = sx / sw; c0[1] = sy / sw;
  }
  const double tf = O_TIE_REL * N;
  o_vtx v[4];
  for (int i = 0; i <= d; ++i) {
    o_vtx w;
    for (int a = 0; a < 3; ++a) w.p[a] = c0[a];
    if (i > 0) w.p[i - 1] = c0[i - 1] + S->step0[i - 1];
    w.f = o_node_eval(L, &C, n, N, w.p[0], w.p[1], w.p[2]).stat;
    o_sx_insert(v, i, w, tf);
  }
  int it = 0, nev = d + 1;
  for (;;) {
    int conv = 1;
    for (int i = 1; i <= d; ++i)
      for (int a = 0; a < d; ++a)
        if (fabs(v[i].p[a] - v[0].p[a]) > S->tol) conv = 0;
    if (conv) break;
    if (!(v[0].f < INFINITY)) { *status |= O_NO_VALID_NODE; break; }
    if (it >= S->max_iter) break;
    ++it;
    /* centroid of the d best vertices */
    double c[3];
    for (int a = 0; a < 3; ++a) {
      double s = 0.0;
      for (int i = 0; i < d; ++i) s += v[i].p[a];
      c[a] = (a < d) ? s / (double)d : v[0].p[a];
    }
    o_vtx r, acc;
    int shrink = 0;
    for (int a = 0; a < 3; ++a) r.p[a] = (a < d) ? c[a] + (c[a] - v[d].p[a]) : c[a];
    r.f = o_node_eval(L, &C, n, N, r.p[0], r.p[1], r.p[2]).stat;
    ++nev;
    if (!o_lt(r.f, v[0].f, tf) && o_lt(r.f, v[d - 1].f, tf)) {
      acc = r;                                       /* reflection */
    } else if (o_lt(r.f, v[0].f, tf)) {
      o_vtx e;                                       /* expansion */
      for (int a = 0; a < 3; ++a) e.p[a] = (a < d) ? c[a] + 2.0 * (r.p[a] - c[a]) : c[a];
      e.f = o_node_eval(L, &C, n, N, e.p[0], e.p[1], e.p[2]).stat;
      ++nev;
      acc = o_lt(e.f, r.f, tf) ? e : r;
    } else if (o_lt(r.f, v[d].f, tf)) {
      o_vtx k;                                       /* outside contraction */
      for (int a = 0; a < 3; ++a) k.p[a] = (a < d) ? c[a] + 0.5 * (r.p[a] - c[a]) : c[a];
      k.f = o_node_eval(L, &C, n, N, k.p[0], k.p[1], k.p[2]).stat;
      ++nev;
      if (!o_lt(r.f, k.f, tf)) acc = k; else shrink = 1;
    } else {
      o_vtx k;                                       /* inside contraction */
      for (int a = 0; a < 3; ++a) k.p[a] = (a < d) ? c[a] + 0.5 * (v[d].p[a] - c[a]) : c[a];
      k.f = o_node_eval(L, &C, n, N, k.p[0], k.p[1], k.p[2]).stat;
      ++nev;
      if (o_lt(k.f, v[d].f, tf)) acc = k; else shrink = 1;
    }
    if (!shrink) {
      o_sx_insert(v, d, acc, tf);
    } else {
      o_vtx w[4];
      w[0] = v[0];
      for (int i = 1; i <= d; ++i) {
        for (int a = 0; a < 3; ++a)
          w[i].p[a] = (a < d) ? v[0].p[a] + 0.5 * (v[i].p[a] - v[0].p[a]) : v[0].p[a];
        w[i].f = o_node_eval(L, &C, n, N, w[i].p[0], w[i].p[1], w[i].p[2]).stat;
        ++nev;
      }
      v[0] = w[0];
      for (int i = 1; i <= d; ++i) o_sx_insert(v, i, w[i], tf);
    }
  }
  *iters = it;
  *evals = nev;
  o_node fin = o_node_eval(L, &C, n, N, v[0].p[0], v[0].p[1], v[0].p[2]);
  out[0] = v[0].p[0]; out[1] = v[0].p[1]; out[2] = v[0].p[2];
  out[3] = fin.A; out[4] = fin.lnl; out[5] = fin.chi2;
  if (!(fin.S > 0.0)) *status |= O_NO_VALID_NODE;
}

void o_reconstruct_simplex(const o_lrf* L, const o_scfg* S, int64_t n_ev, const double* sig,
                           const double* seeds, double* out6, int* ndf, int* status, int* iters,
                           int* evals, int n_threads) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
  for (int64_t e = 0; e < n_ev; ++e)
    o_simplex_event(L, S, sig + e * L->n_sensors, seeds ? seeds + 4 * e : NULL, out6 + 6 * e,
                    ndf + e, status + e, iters + e, evals + e);
}

/* ------------------------------------------------------------------ */
/* Variable-metric search per event (Sec. 5.1.2.1: the Minuit2 Migrad    */
/* minimiser, a variable-metric method with numerical derivatives, over  */
/* x, y or x, y, z from the centroid, the strongest sensor or a seed).   */
/* The statistic is the grid's node statistic (ML or chi2, energy from   */
/* the ratio of the sums).  Readings (the paper names the library, not   */
/* its steps; written from the textbook quasi-Newton method):            */
/*  - gradient g by central differences with step h (mm) per searched    */
/*    axis: g_a = (F(p + h e_a) - F(p - h e_a)) / (2 h);                  */
/*  - initial inverse curvature V diagonal: V_aa = 1 / d2_a with          */
/*    d2_a = (F(p + h e_a) - 2 F(p) + F(p - h e_a)) / h^2 from the same    */
/*    points, or step0_a^2 where d2_a is not positive and finite;        */
/*  - estimated distance to the minimum EDM = g^T V g / 2; stop when      */
/*    EDM < edm_tol, or after max_iter iterations;                        */
/*  - direction d = -V g; if g^T d >= 0, V is reset to diag(step0^2);     */
/*    if still g^T d >= 0, stop;                                          */
/*  - line search: alpha = 1, halved (at most 20 times) until            */
/*    F(p + alpha d) <= F(p) + 1e-4 alpha g^T d; no such alpha: stop;     */
/*  - BFGS update of V with s = p' - p, y = g' - g when s^T y > 0:       */
/*    V' = V + (s^T y + y^T V y) / (s^T y)^2 s s^T                        */
/*           - (V y s^T + s y^T V) / (s^T y);                             */
/*  - a start where F is not finite gives NO_VALID_NODE (the start is    */
/*    reported); a non-finite gradient ends the search at the current    */
/*    point (at the start, before any step);                              */
/*  - coordinates that are arguments of the LRF's splines are limited to */
/*    the spline's domain [lo, hi] as Minuit limits parameters: the       */
/*    search runs in an internal coordinate u with the position            */
/*    lo + (hi - lo) (sin u + 1) / 2 (z for r-z and sliced LRFs, x and y  */
/*    for XY and sliced LRFs); the start enters as u = asin(2 (p - lo) /   */
/*    (hi - lo) - 1) (clamped into the domain), the difference step and   */
/*    the fallback scale are divided by (hi - lo) / 2.  Beyond such a     */
/*    wall the statistic jumps to infinity; in u the wall is a smooth     */
/*    turning point, so searches that end against it stop reproducibly.  */
/* An iteration is one accepted step.  Arithmetic as written (no fused   */
/* multiply-add), sums in axis order.                                    */
/* ------------------------------------------------------------------ */
typedef struct {
  int dims;             /* 2: x, y;  3: x, y, z                          */
  int stat;             /* 0 ML, 1 chi2                                  */
  int start;            /* 0 CoG, 1 strongest sensor, 2 seed             */
  double step0[3];      /* scale per axis (mm): fallback curvature        */
  double z_start;
  double h;             /* central-difference step (mm)                   */
  double edm_tol;       /* stop when EDM < edm_tol                        */
  int max_iter;
  double l_floor, v_floor;
} o_vcfg;

static double o_vm_f(const o_lrf* L, const o_cfg* C, const double* n, double N, const double p[3],
                     int* nev) {
  ++*nev;
  double f = o_node_eval(L, C, n, N, p[0], p[1], p[2]).stat;
  return isfinite(f) ? f : INFINITY;
}

/* central-difference gradient and curvature estimates at internal point u
 * (statistic f there), steps hs per axis; returns 0 when a value is not
 * finite */
static void o_vm_ext(const o_lrf* L, int d, const double u[3], const double z_start, double p[3]);
static int o_vm_grad(const o_lrf* L, const o_cfg* C, const double* n, double N, const double u[3],
                     double f, int d, const double hs[3], double z_start, double g[3],
                     double d2[3], int* nev) {
  for (int a = 0; a < 3; ++a) { g[a] = 0.0; d2[a] = 0.0; }
  for (int a = 0; a < d; ++a) {
    double q[3] = {u[0], u[1], u[2]}, x[3];
    q[a] = u[a] + hs[a];
    o_vm_ext(L, d, q, z_start, x);
    const double fp = o_vm_f(L, C, n, N, x, nev);
    q[a] = u[a] - hs[a];
    o_vm_ext(L, d, q, z_start, x);
    const double fm = o_vm_f(L, C, n, N, x, nev);
    if (!isfinite(fp) || !isfinite(fm)) return 0;
    g[a] = (fp - fm) / (2.0 * hs[a]);
    d2[a] = ((fp - 2.0 * f) + fm) / (hs[a] * hs[a]);
  }
  return 1;
}

/* limits of searched axis a (0 x, 1 y, 2 z) from the LRF's spline domain */
static int o_vm_limit(const o_lrf* L, int a, double* lo, double* hi) {
  if (a == 2 && (L->kind == 3 || L->kind == 5)) {
    *lo = L->kind == 3 ? L->lo[1] : L->z_lo;
    *hi = L->kind == 3 ? L->hi[1] : L->z_hi;
    return 1;
  }
  if (a < 2 && (L->kind == 2 || L->kind == 5)) {
    *lo = L->lo[a];
    *hi = L->hi[a];
    return 1;
  }
  return 0;
}

/* position of internal point u (limited axes transformed) */
static void o_vm_ext(const o_lrf* L, int d, const double u[3], const double z_start, double p[3]) {
  p[0] = u[0]; p[1] = u[1]; p[2] = d == 3 ? u[2] : z_start;
  for (int a = 0; a < d; ++a) {
    double lo, hi;
    if (o_vm_limit(L, a, &lo, &hi)) p[a] = lo + (0.5 * (hi - lo)) * (sin(u[a]) + 1.0);
  }
}

void o_migrad_event(const o_lrf* L, const o_vcfg* S, const double* n, const double* seed,
                    double out[6], int* ndf, int* status, int* iters, int* evals) {
  int ns = L->n_sensors, na = 0, bad = 0, d = S->dims;
  double N = 0.0;
  *status = 0;
  *iters = 0;
  *evals = 0;
  for (int i = 0; i < ns; ++i) {
    if (!L->active[i]) continue;
    ++na;
    if (!isfinite(n[i]) || n[i] < 0.0) bad = 1;
    else N += n[i];
  }
  *ndf = na - (d + 1);
  for (int k = 0; k < 6; ++k) out[k] = NAN;
  if (na == 0) { *status = O_NO_ACTIVE; return; }
  if (bad) { *status = O_BAD_INPUT; return; }
  if (!(N > 0.0)) { *status = O_EMPTY; return; }
  o_cfg C;
  memset(&C, 0, sizeof(C));
  C.stat = S->stat;
  C.l_floor = S->l_floor;
  C.v_floor = S->v_floor;
  double p[3] = {0.0, 0.0, S->z_start};
  if (S->start == 2 && seed) {
    p[0] = seed[0]; p[1] = seed[1];
    if (d == 3) p[2] = seed[2];
  } else if (S->start == 1) {
    int best = -1;
    for (int i = 0; i < ns; ++i)
      if (L->active[i] && (best < 0 || n[i] > n[best])) best = i;
    p[0] = L->sxy[2 * best]; p[1] = L->sxy[2 * best + 1];
  } else {
    double sw = 0.0, sx = 0.0, sy = 0.0;
    for (int i = 0; i < ns; ++i) {
      if (!L->active[i]) continue;
      double w = n[i] / L->gain[i];
      sw += w; sx += L->sxy[2 * i] * w; sy += L->sxy[2 * i + 1] * w;
    }
    p[0] = sx / sw; p[1] = sy / sw;
  }
  /* internal coordinates, difference steps and fallback scales */
  double u[3] = {p[0], p[1], p[2]}, hs[3], s0[3];
  for (int a = 0; a < 3; ++a) { hs[a] = S->h; s0[a] = S->step0[a]; }
  for (int a = 0; a < d; ++a) {
    double lo, hi;
    if (!o_vm_limit(L, a, &lo, &hi)) continue;
    const double half = 0.5 * (hi - lo);
    double w = (p[a] - lo) / half - 1.0;
    w = w < -1.0 ? -1.0 : w > 1.0 ? 1.0 : w;
    u[a] = asin(w);
    hs[a] = S->h / half;
    s0[a] = S->step0[a] / half;
  }
  int nev = 0, it = 0;
  double q[3];
  o_vm_ext(L, d, u, S->z_start, q);
  double f = o_vm_f(L, &C, n, N, q, &nev);
  double g[3], d2[3], V[3][3];
  if (isfinite(f) && o_vm_grad(L, &C, n, N, u, f, d, hs, S->z_start, g, d2, &nev)) {
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) V[a][b] = 0.0;
    for (int a = 0; a < d; ++a)
      V[a][a] = (d2[a] > 0.0 && isfinite(d2[a])) ? 1.0 / d2[a] : s0[a] * s0[a];
    while (it < S->max_iter) {
      /* EDM = g^T V g / 2, direction -V g, slope g^T dir */
      double Vg[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) Vg[a] += V[a][b] * g[b];
      double edm = 0.0;
      for (int a = 0; a < d; ++a) edm += g[a] * Vg[a];
      edm = 0.5 * edm;
      if (edm < S->edm_tol) break;
      double dir[3] = {0.0, 0.0, 0.0}, slope = 0.0;
      for (int a = 0; a < d; ++a) { dir[a] = -Vg[a]; slope += g[a] * dir[a]; }
      if (!(slope < 0.0)) {
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) V[a][b] = (a == b) ? s0[a] * s0[a] : 0.0;
        slope = 0.0;
        for (int a = 0; a < d; ++a) { dir[a] = -(V[a][a] * g[a]); slope += g[a] * dir[a]; }
        if (!(slope < 0.0)) break;
      }
      double alpha = 1.0, ut[3] = {u[0], u[1], u[2]}, ft = INFINITY;
      int ok = 0;
      for (int ls = 0; ls <= 20; ++ls) {
        for (int a = 0; a < d; ++a) ut[a] = u[a] + alpha * dir[a];
        o_vm_ext(L, d, ut, S->z_start, q);
        ft = o_vm_f(L, &C, n, N, q, &nev);
        if (ft <= f + 1e-4 * alpha * slope) { ok = 1; break; }
        alpha = 0.5 * alpha;
      }
      if (!ok) break;
      double gn[3], d2n[3];
      const int gok = o_vm_grad(L, &C, n, N, ut, ft, d, hs, S->z_start, gn, d2n, &nev);
      double sv[3] = {0.0, 0.0, 0.0}, yv[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < d; ++a) { sv[a] = ut[a] - u[a]; yv[a] = gn[a] - g[a]; }
      for (int a = 0; a < 3; ++a) u[a] = ut[a];
      f = ft;
      ++it;
      if (!gok) break;
      double sy = 0.0;
      for (int a = 0; a < d; ++a) sy += sv[a] * yv[a];
      if (sy > 0.0) {
        double Vy[3] = {0.0, 0.0, 0.0}, yVy = 0.0;
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b) Vy[a] += V[a][b] * yv[b];
        for (int a = 0; a < d; ++a) yVy += yv[a] * Vy[a];
        const double c1 = (sy + yVy) / (sy * sy);
        for (int a = 0; a < d; ++a)
          for (int b = 0; b < d; ++b)
            V[a][b] = (V[a][b] + c1 * (sv[a] * sv[b])) - (Vy[a] * sv[b] + sv[a] * Vy[b]) / sy;
      }
      for (int a = 0; a < 3; ++a) g[a] = gn[a];
    }
  }
  o_vm_ext(L, d, u, S->z_start, p);
  *iters = it;
  *evals = nev;
  o_node fin = o_node_eval(L, &C, n, N, p[0], p[1], p[2]);
  out[0] = p[0]; out[1] = p[1]; out[2] = p[2];
  out[3] = fin.A; out[4] = fin.lnl; out[5] = fin.chi2;
  if (!isfinite(f) || !(fin.S > 0.0)) *status |= O_NO_VALID_NODE;
}

void o_reconstruct_migrad(const o_lrf* L, const o_vcfg* S, int64_t n_ev, const double* sig,
                          const double* seeds, double* out6, int* ndf, int* status, int* iters,
                          int* evals, int n_threads) {
#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
  for (int64_t e = 0; e < n_ev; ++e)
    o_migrad_event(L, S, sig + e * L->n_sensors, seeds ? seeds + 4 * e : NULL, out6 + 6 * e,
                   ndf + e, status + e, iters + e, evals + e);
}

/* ------------------------------------------------------------------ */
/* k-NN reconstruction (Sec. 5.1.4): each event is a point whose        */
/* coordinates are the normalised signals of the sensors; the position  */
/* is the centroid of the known positions of the k calibration events   */
/* closest to it.  Readings:                                            */
/*  - normalised signal of active sensor i: n_i / N, N = sum over the    */
/*    active sensors (in sensor order), divided in double precision and */
/*    rounded to single precision;                                      */
/*  - distance: squared Euclidean over the active sensors, accumulated  */
/*    in sensor order in single precision with each subtraction,        */
/*    square and sum rounded as written.  The distance decides which    */
/*    events are neighbours (an integer result), so it is defined in    */
/*    the precision the GPU kernel computes it in;                      */
/*  - order: (distance, calibration index), the lower index first on    */
/*    equal distances; the k first are the neighbours;                  */
/*  - calibration events with N <= 0 or a non-finite or negative active */
/*    signal never become neighbours; a query with such signals gets    */
/*    NaN and the grid's status bits;                                   */
/*  - position: the mean of the k (or fewer, if fewer calibration       */
/*    events are valid) neighbours' positions, summed in double in      */
/*    neighbour order.                                                  */
/* ------------------------------------------------------------------ */

/* normalised signals of one event: q[na]; returns the status bits */
static int o_knn_norm(const o_lrf* L, const double* n, float* q) {
  int na = 0, bad = 0;
  double N = 0.0;
  for (int i = 0; i < L->n_sensors; ++i) {
    if (!L->active[i]) continue;
    ++na;
    if (!isfinite(n[i]) || n[i] < 0.0) bad = 1;
    else N += n[i];
  }
  if (na == 0) return O_NO_ACTIVE;
  if (bad) return O_BAD_INPUT;
  if (!(N > 0.0)) return O_EMPTY;
  int a = 0;
  for (int i = 0; i < L->n_sensors; ++i)
    if (L->active[i]) q[a++] = (float)(n[i] / N);
  return 0;
}

static float o_knn_dist(const float* q, const float* c, int na) {
  float s = 0.0f;
  for (int a = 0; a < na; ++a) {
    float d = q[a] - c[a];
    float d2 = d * d;
    s = s + d2;
  }
  return s;
}

typedef struct { float d; int64_t i; } o_nb;

static int o_nb_cmp(const void* A, const void* B) {
  const o_nb* a = (const o_nb*)A;
  const o_nb* b = (const o_nb*)B;
  if (a->d < b->d) return -1;
  if (a->d > b->d) return 1;
  return (a->i > b->i) - (a->i < b->i);
}

/* Normalised calibration points [m][na] (rows of invalid events are
 * flagged in valid[]). */
void o_knn_prepare(const o_lrf* L, int64_t m, const double* sig, float* cal, uint8_t* valid,
                   int n_threads) {
  int na = 0;
  for (int i = 0; i < L->n_sensors; ++i) na += L->active[i] != 0;
#pragma omp parallel for schedule(static) num_threads(n_threads)
  for (int64_t c = 0; c < m; ++c)
    valid[c] = o_knn_norm(L, sig + c * L->n_sensors, cal + c * na) == 0;
}

/* Queries: out3 [n][3] positions, status [n], nb_idx / nb_dist [n][k] the
 * neighbours in order (-1 / +inf past the valid ones). */
void o_knn_reconstruct(const o_lrf* L, int64_t m, const float* cal, const uint8_t* valid,
                       const double* cal_pos /* [m][3] */, int k, int64_t n, const double* sig,
                       double* out3, int* status, int64_t* nb_idx, float* nb_dist,
                       int n_threads) {
  int na = 0;
  for (int i = 0; i < L->n_sensors; ++i) na += L->active[i] != 0;
#pragma omp parallel for schedule(dynamic, 4) num_threads(n_threads)
  for (int64_t e = 0; e < n; ++e) {
    float* q = (float*)malloc(sizeof(float) * (size_t)(na > 0 ? na : 1));
    o_nb* all = (o_nb*)malloc(sizeof(o_nb) * (size_t)(m > 0 ? m : 1));
    for (int a = 0; a < 3; ++a) out3[3 * e + a] = NAN;
    for (int j = 0; j < k; ++j) { nb_idx[e * k + j] = -1; nb_dist[e * k + j] = INFINITY; }
    status[e] = o_knn_norm(L, sig + e * L->n_sensors, q);
    if (status[e] == 0) {
      int64_t cnt = 0;
      for (int64_t c = 0; c < m; ++c) {
        if (!valid[c]) continue;
        all[cnt].d = o_knn_dist(q, cal + c * na, na);
        all[cnt].i = c;
        ++cnt;
      }
      qsort(all, (size_t)cnt, sizeof(o_nb), o_nb_cmp);
      int kk = cnt < k ? (int)cnt : k;
      double s[3] = {0.0, 0.0, 0.0};
      for (int j = 0; j < kk; ++j) {
        nb_idx[e * k + j] = all[j].i;
        nb_dist[e * k + j] = all[j].d;
        for (int a = 0; a < 3; ++a) s[a] += cal_pos[3 * all[j].i + a];
      }
      if (kk > 0)
        for (int a = 0; a < 3; ++a) out3[3 * e + a] = s[a] / (double)kk;
      else
        status[e] = O_NO_VALID_NODE;
    }
    free(q);
    free(all);
  }
}
