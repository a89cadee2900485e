// Two-dimensional LRF fits from events (the LRF module, Sec. 6: r-z LRFs
// in r and depth, and per-sensor XY LRFs in the detector plane, Sec.
// 6.1.1; sensor groups sharing one LRF, Sec. 6.2; alternated with the
// reconstruction by the iterative procedure, Sec. 8).
//
// Least squares on the estimates n / (E g) of L(u, w), one per (event,
// sensor) pair with both spline arguments in their domains, on the
// reconstruction's tensor-product cubic B-spline (table [nb1 + 2][nb0 + 2],
// coefficient index j1 (nb0 + 2) + j0).  A pair touches a 4 x 4 patch of
// coefficients, so a group's normal matrix is banded with half width
// 3 (nb0 + 2) + 3 in that index; it is accumulated in FP64 in global memory
// (the pair's 136 products and 16 right-side terms by atomic adds: sums in
// arrival order, so the last bits may differ from call to call), then one
// wave per group adds the relative ridge and solves by banded Cholesky.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "ants_internal.h"
#include "lrf64.h"

using namespace ants;

namespace {

constexpr int kFit2MaxKnots = 64;
constexpr int kFit2MaxGroups = 1024;

struct Fit2P {
  const int32_t* col;
  const double *X, *Y, *g;
  int na;
  const float* sig;
  int64_t ld, n;
  const float *x, *y, *z, *E, *chi2;
  const int32_t *ndf, *status;
  const float* shift;
  double chi2ndf_max;
  int rz;              // 1: arguments (r, z); 0: (x, y)
  int nb0, nb1, nc0, nc, bw;
  double lo0, hi0, lo1, hi1, inv_d0, inv_d1;
  const int32_t* group;   // per sensor index
  int groups;
  double* band;        // [groups][nc][bw + 1]: entry (i, i + k) at [i][k]
  double* rhs;         // [groups][nc]
  unsigned long long* pairs;   // [groups]
  unsigned long long* used;    // [1]
};

__global__ void fit2_zero_kernel(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// one wave per event at a time, lanes over the active sensors
__global__ void __launch_bounds__(256) fit2_accum_kernel(Fit2P P) {
  const int lane = threadIdx.x & 63;
  const int64_t w0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int nc0 = P.nc0, bw = P.bw;
  for (int64_t e = w0; e < P.n; e += nw) {
    const float Ef = P.E[e];
    bool ok = (P.status[e] & kEvFailed) == 0 && Ef > 0.f && Ef < __builtin_huge_valf();
    if (P.chi2ndf_max > 0.0) {
      const int d = P.ndf[e];
      ok = ok && d > 0 && (double)P.chi2[e] / (double)d <= P.chi2ndf_max;
    }
    if (!ok) continue;   // uniform over the wave
    if (lane == 0) atomicAdd(P.used, 1ull);
    double xe = P.x[e], ye = P.y[e];
    if (P.shift) {
      xe += (double)P.shift[2 * e];
      ye += (double)P.shift[2 * e + 1];
    }
    const double ze = P.z[e], Ee = Ef;
    const float* row = P.sig + e * P.ld;
    for (int a = lane; a < P.na; a += 64) {
      const int gr = P.group[P.col[a]];
      if (gr < 0 || gr >= P.groups) continue;
      double u, w;
      if (P.rz) {
        const double dx = xe - P.X[a], dy = ye - P.Y[a];
        u = sqrt(dx * dx + dy * dy);
        w = ze;
      } else {
        u = xe;
        w = ye;
      }
      int m0, m1;
      double t0, t1;
      if (!locate64(u, P.nb0, P.lo0, P.hi0, P.inv_d0, m0, t0)) continue;
      if (!locate64(w, P.nb1, P.lo1, P.hi1, P.inv_d1, m1, t1)) continue;
      double b0[4], b1[4];
      bweights64(t0, b0);
      bweights64(t1, b1);
      const double tg = (double)row[P.col[a]] / (Ee * P.g[a]);
      double* band = P.band + (int64_t)gr * P.nc * (bw + 1);
      double* rhs = P.rhs + (int64_t)gr * P.nc;
      int idx[16];
      double wt[16];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          idx[4 * q + p] = (m1 + q) * nc0 + (m0 + p);
          wt[4 * q + p] = b1[q] * b0[p];
        }
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        atomicAdd(&rhs[idx[i]], wt[i] * tg);
#pragma unroll
        for (int j = i; j < 16; ++j)   // idx increases with (q, p): idx[j] >= idx[i]
          atomicAdd(&band[(int64_t)idx[i] * (bw + 1) + (idx[j] - idx[i])], wt[i] * wt[j]);
      }
      atomicAdd(&P.pairs[gr], 1ull);
    }
  }
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

struct Solve2P {
  double* band;
  const double* rhs;
  int nc, bw, nc0, nc1;
  double ridge;
  double* y;           // [groups][nc] work
  double* coef;        // [groups][nc1][nc0]
  int64_t* counts;     // [groups][2] or NULL
  const unsigned long long *pairs, *used;
};

// one wave per group: ridge * mean diagonal on the diagonal, U^T U = A
// (U upper, in place of the band), then U^T y = v and U c = y
__global__ void __launch_bounds__(64) fit2_solve_kernel(Solve2P P) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x, gr = blockIdx.x;
  const int nc = P.nc, bw = P.bw, W = bw + 1;
  double* U = P.band + (int64_t)gr * nc * W;
  const double* v = P.rhs + (int64_t)gr * nc;
  double* y = P.y + (int64_t)gr * nc;
  double tr = 0.0;
  for (int i = lane; i < nc; i += 64) tr += U[(int64_t)i * W];
  tr = wave_sum(tr);
  const double lam = P.ridge * (tr / nc);
  for (int i = lane; i < nc; i += 64) U[(int64_t)i * W] += lam;
  __syncthreads();
  for (int j = 0; j < nc; ++j) {
    const int k0 = j - bw > 0 ? j - bw : 0;
    double s = 0.0;
    for (int k = k0 + lane; k < j; k += 64) {
      const double u = U[(int64_t)k * W + (j - k)];
      s += u * u;
    }
    s = wave_sum(s);
    const double dj = U[(int64_t)j * W] - s;
    const double d = dj > 0.0 ? sqrt(dj) : __builtin_nan("");
    __syncthreads();
    if (lane == 0) U[(int64_t)j * W] = d;
    const int i1 = j + bw < nc - 1 ? j + bw : nc - 1;
    for (int i = j + 1 + lane; i <= i1; i += 64) {
      const int kk = i - bw > 0 ? i - bw : 0;
      double t = U[(int64_t)j * W + (i - j)];
      for (int k = kk > k0 ? kk : k0; k < j; ++k)
        t -= U[(int64_t)k * W + (j - k)] * U[(int64_t)k * W + (i - k)];
      U[(int64_t)j * W + (i - j)] = t / d;
    }
    __syncthreads();
  }
  // U^T y = v (forward), then U c = y (backward)
  for (int j = 0; j < nc; ++j) {
    const int k0 = j - bw > 0 ? j - bw : 0;
    double s = 0.0;
    for (int k = k0 + lane; k < j; k += 64) s += U[(int64_t)k * W + (j - k)] * y[k];
    s = wave_sum(s);
    __syncthreads();
    if (lane == 0) y[j] = (v[j] - s) / U[(int64_t)j * W];
    __syncthreads();
  }
  double* c = P.coef + (int64_t)gr * nc;
  for (int j = nc - 1; j >= 0; --j) {
    const int i1 = j + bw < nc - 1 ? j + bw : nc - 1;
    double s = 0.0;
    for (int i = j + 1 + lane; i <= i1; i += 64) s += U[(int64_t)j * W + (i - j)] * c[i];
    s = wave_sum(s);
    __syncthreads();
    if (lane == 0) c[j] = (y[j] - s) / U[(int64_t)j * W];
    __syncthreads();
  }
  if (P.counts && lane == 0) {
    P.counts[2 * gr] = (int64_t)*P.used;
    P.counts[2 * gr + 1] = (int64_t)P.pairs[gr];
  }
}

}  // namespace

extern "C" ants_status ants_fit_lrf2d_grouped(ants_lrfset* set, const ants_fit2d_cfg* cfg,
                                              int32_t n_groups, const int32_t* d_group,
                                              int64_t n_events, const float* d_signals,
                                              int64_t ld, ants_out rec, const float* d_shift,
                                              double* d_coef, int64_t* d_counts,
                                              void* hip_stream) {
  const char* who = "ants_fit_lrf2d_grouped";
  if (!set || !cfg || !d_coef || !d_group) return set_error(ANTS_E_ARG, "%s: NULL argument", who);
  if (cfg->kind != ANTS_LRF_RZ && cfg->kind != ANTS_LRF_XY)
    return set_error(ANTS_E_ARG, "%s: kind %d must be r-z or XY", who, cfg->kind);
  for (int a = 0; a < 2; ++a) {
    if (cfg->nb[a] < 4 || cfg->nb[a] > kFit2MaxKnots)
      return set_error(ANTS_E_ARG, "%s: nb[%d] = %d outside 4..%d", who, a, cfg->nb[a],
                       kFit2MaxKnots);
    if (!(cfg->hi[a] > cfg->lo[a] && isfinite(cfg->lo[a]) && isfinite(cfg->hi[a])))
      return set_error(ANTS_E_ARG, "%s: domain %d [%g, %g] invalid", who, a, cfg->lo[a],
                       cfg->hi[a]);
  }
  if (cfg->kind == ANTS_LRF_RZ && cfg->lo[0] < 0.0)
    return set_error(ANTS_E_ARG, "%s: an r domain starts at r >= 0", who);
  if (!(cfg->ridge >= 0.0 && cfg->ridge < 1e300))
    return set_error(ANTS_E_ARG, "%s: ridge %g invalid", who, cfg->ridge);
  if (n_groups < 1 || n_groups > kFit2MaxGroups)
    return set_error(ANTS_E_ARG, "%s: %d groups outside 1..%d", who, n_groups, kFit2MaxGroups);
  if (n_events < 0) return set_error(ANTS_E_ARG, "%s: n_events < 0", who);
  if (n_events > 0 && (!d_signals || !rec.x || !rec.y || !rec.z || !rec.E || !rec.chi2 ||
                       !rec.ndf || !rec.status))
    return set_error(ANTS_E_ARG, "%s: NULL signals or reconstruction field", who);
  if (ld < set->ns) return set_error(ANTS_E_ARG, "%s: ld < n_sensors", who);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || set->device != dev)
    return set_error(ANTS_E_ARG, "%s: set on another device", who);
  const int nc0 = cfg->nb[0] + 2, nc1 = cfg->nb[1] + 2, nc = nc0 * nc1, bw = 3 * nc0 + 3;
  const size_t nband = (size_t)n_groups * nc * (bw + 1), nrhs = (size_t)n_groups * nc;
  const size_t bytes = (nband + 2 * nrhs) * sizeof(double) +
                       ((size_t)n_groups + 1) * sizeof(unsigned long long);
  hipError_t e = ensure(&set->ws_fit2, &set->ws_fit2_bytes, bytes);
  if (e != hipSuccess) return hip_error(e, who);
  double* band = (double*)set->ws_fit2;
  double* rhs = band + nband;
  double* ywork = rhs + nrhs;
  unsigned long long* pairs = (unsigned long long*)(ywork + nrhs);
  unsigned long long* used = pairs + n_groups;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t nz = (int64_t)(bytes / sizeof(double));
  hipLaunchKernelGGL(fit2_zero_kernel, dim3((unsigned)std::min<int64_t>((nz + 255) / 256, 4096)),
                     dim3(256), 0, s, (double*)set->ws_fit2, nz);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, who);
  if (n_events > 0) {
    Fit2P P;
    memset(&P, 0, sizeof(P));
    P.col = set->d.col;
    P.X = set->d.X;
    P.Y = set->d.Y;
    P.g = set->d.g;
    P.na = set->d.na;
    P.sig = d_signals;
    P.ld = ld;
    P.n = n_events;
    P.x = rec.x;
    P.y = rec.y;
    P.z = rec.z;
    P.E = rec.E;
    P.chi2 = rec.chi2;
    P.ndf = rec.ndf;
    P.status = rec.status;
    P.shift = d_shift;
    P.chi2ndf_max = cfg->chi2ndf_max;
    P.rz = cfg->kind == ANTS_LRF_RZ;
    P.nb0 = cfg->nb[0];
    P.nb1 = cfg->nb[1];
    P.nc0 = nc0;
    P.nc = nc;
    P.bw = bw;
    P.lo0 = cfg->lo[0];
    P.hi0 = cfg->hi[0];
    P.lo1 = cfg->lo[1];
    P.hi1 = cfg->hi[1];
    P.inv_d0 = (double)(cfg->nb[0] - 1) / (cfg->hi[0] - cfg->lo[0]);
    P.inv_d1 = (double)(cfg->nb[1] - 1) / (cfg->hi[1] - cfg->lo[1]);
    P.group = d_group;
    P.groups = n_groups;
    P.band = band;
    P.rhs = rhs;
    P.pairs = pairs;
    P.used = used;
    int64_t blocks = (n_events + 3) / 4;
    const int64_t cap = (int64_t)num_cu() * 8;
    if (blocks > cap) blocks = cap;
    hipLaunchKernelGGL(fit2_accum_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, who);
  }
  Solve2P S;
  S.band = band;
  S.rhs = rhs;
  S.nc = nc;
  S.bw = bw;
  S.nc0 = nc0;
  S.nc1 = nc1;
  S.ridge = cfg->ridge;
  S.y = ywork;
  S.coef = d_coef;
  S.counts = d_counts;
  S.pairs = pairs;
  S.used = used;
  hipLaunchKernelGGL(fit2_solve_kernel, dim3(n_groups), dim3(64), 0, s, S);
  e = hipGetLastError();
  return e == hipSuccess ? ANTS_OK : hip_error(e, who);
}
