// LRF fit from events (the LRF module computing LRFs from signals and event
// positions, Sec. 6; one LRF for all sensors with relative gains, Sec. 6.2;
// alternated with the reconstruction by the iterative procedure, Sec. 8).
//
// Axial LRF, one shared cubic B-spline table of nc = nb + 2 coefficients:
// least squares on the estimates n / (E g) of L(r), one per (event, active
// sensor) pair inside the domain.  The normal matrix is banded (a pair
// touches four consecutive coefficients), so each wave accumulates its band
// (4 diagonals) and right-hand side in FP64 in its own LDS area; the waves'
// partial sums are added by a fixed tree and one wave solves the system by
// Cholesky.  Results do not depend on the launch's timing.
#include <math.h>
#include <string.h>

#include "ants_internal.h"
#include "lrf64.h"

using namespace ants;

namespace {

constexpr int kFitMaxCoef = 64;
constexpr int kFitWaves = 4;   // waves per block of the accumulation
constexpr int kFitCopies = 4;  // accumulator copies per wave (lane % 4), fewer same-address atomics

struct FitP {
  const int32_t* col;
  const double *X, *Y, *g;
  int na;
  const float* sig;
  int64_t ld, n;
  const float *x, *y, *E, *chi2;
  const int32_t *ndf, *status;
  double chi2ndf_max;
  int nb, nc;
  double lo, hi, inv_d;
  double* part;      // [waves][nc * 5 + 2]: band (row-major, 4 diagonals), rhs, counts
  int stride;
};

__global__ void __launch_bounds__(64 * kFitWaves) fit_accum_kernel(FitP P) {
  extern __shared__ double fsm[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nc = P.nc;
  double* wacc = fsm + wv * (nc * 5 * kFitCopies);
  double* acc = wacc + (lane % kFitCopies) * (nc * 5);
  for (int i = lane; i < nc * 5 * kFitCopies; i += 64) wacc[i] = 0.0;
  __syncthreads();
  const int64_t gw = (int64_t)blockIdx.x * kFitWaves + wv;
  const int64_t nw = (int64_t)gridDim.x * kFitWaves;
  double used = 0.0, pairs = 0.0;
  for (int64_t e = gw; e < P.n; e += nw) {
    const float Ef = P.E[e];
    bool ok = P.status[e] == 0 && Ef > 0.f && Ef < __builtin_huge_valf();
    if (P.chi2ndf_max > 0.0) {
      const int d = P.ndf[e];
      ok = ok && d > 0 && (double)P.chi2[e] / (double)d <= P.chi2ndf_max;
    }
    if (!ok) continue;   // uniform over the wave
    used += 1.0;
    const double xe = P.x[e], ye = P.y[e], Ee = Ef;
    const float* row = P.sig + e * P.ld;
    for (int a = lane; a < P.na; a += 64) {
      const double dx = xe - P.X[a], dy = ye - P.Y[a];
      const double r = sqrt(dx * dx + dy * dy);
      int m;
      double t;
      if (!locate64(r, P.nb, P.lo, P.hi, P.inv_d, m, t)) continue;
      double b[4];
      bweights64(t, b);
      const double tg = (double)row[P.col[a]] / (Ee * P.g[a]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        atomicAdd(&acc[4 * nc + m + k], b[k] * tg);
#pragma unroll
        for (int l = k; l < 4; ++l) atomicAdd(&acc[4 * (m + k) + (l - k)], b[k] * b[l]);
      }
      pairs += 1.0;
    }
  }
  __syncthreads();
  double* out = P.part + gw * P.stride;
  for (int i = lane; i < nc * 5; i += 64) {
    double v = wacc[i];
    for (int c = 1; c < kFitCopies; ++c) v += wacc[c * nc * 5 + i];
    out[i] = v;
  }
  // pair count of the wave (each lane counted its own pairs)
  for (int o = 32; o >= 1; o >>= 1) pairs += __shfl_xor(pairs, o);
  if (lane == 0) {
    out[nc * 5] = used;
    out[nc * 5 + 1] = pairs;
  }
}

// LDS writes of the wave visible to all of its lanes
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SolveP {
  const double* part;
  int stride, nwaves, nc;
  double ridge;
  double* sums;      // [stride]: the waves' partials added up
  double* coef;
  int64_t* counts;
};

// One block per entry of the partials: the waves' values added by a fixed
// tree (thread t takes waves t, t + 256, ...; then pairwise halving).
__global__ void __launch_bounds__(256) fit_reduce_kernel(SolveP P) {
  __shared__ double red[256];
  const int i = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int w = tid; w < P.nwaves; w += 256) s += P.part[(int64_t)w * P.stride + i];
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) P.sums[i] = red[0];
}

__global__ void __launch_bounds__(64) fit_solve_kernel(SolveP P) {
  __shared__ double band[kFitMaxCoef * 5 + 2];
  __shared__ double A[kFitMaxCoef][kFitMaxCoef + 1];
  __shared__ double y[kFitMaxCoef];
  const int lane = threadIdx.x, nc = P.nc;
  for (int i = lane; i < nc * 5 + 2; i += 64) band[i] = P.sums[i];
  wave_sync();
  // dense symmetric matrix from the band, plus the relative ridge
  for (int i = 0; i < nc; ++i)
    for (int j = lane; j < nc; j += 64) {
      const int lo = i < j ? i : j, dd = i < j ? j - i : i - j;
      A[i][j] = dd < 4 ? band[4 * lo + dd] : 0.0;
    }
  wave_sync();
  double tr = 0.0;
  for (int i = 0; i < nc; ++i) tr += A[i][i];
  const double lam = P.ridge * tr / nc;
  if (lane < nc) A[lane][lane] += lam;
  wave_sync();
  // Cholesky A = L L^T, L in the lower triangle (column j by the lanes i >= j)
  for (int j = 0; j < nc; ++j) {
    if (lane == j) {
      double d = A[j][j];
      for (int k = 0; k < j; ++k) d -= A[j][k] * A[j][k];
      A[j][j] = d > 0.0 ? sqrt(d) : __builtin_nan("");
    }
    wave_sync();
    if (lane > j && lane < nc) {
      double s = A[lane][j];
      for (int k = 0; k < j; ++k) s -= A[lane][k] * A[j][k];
      A[lane][j] = s / A[j][j];
    }
    wave_sync();
  }
  // L y = v, then L^T c = y (one lane; nc <= 64)
  if (lane == 0) {
    for (int i = 0; i < nc; ++i) {
      double s = band[4 * nc + i];
      for (int k = 0; k < i; ++k) s -= A[i][k] * y[k];
      y[i] = s / A[i][i];
    }
    for (int i = nc - 1; i >= 0; --i) {
      double s = y[i];
      for (int k = i + 1; k < nc; ++k) s -= A[k][i] * y[k];
      y[i] = s / A[i][i];
    }
    for (int i = 0; i < nc; ++i) P.coef[i] = y[i];
    if (P.counts) {
      P.counts[0] = (int64_t)band[nc * 5];
      P.counts[1] = (int64_t)band[nc * 5 + 1];
    }
  }
}

bool rec_ok(const ants_out& o) { return o.x && o.y && o.E && o.chi2 && o.ndf && o.status; }

}  // namespace

extern "C" ants_status ants_fit_axial_lrf(ants_lrfset* set, const ants_fit_cfg* cfg,
                                          int64_t n_events, const float* d_signals, int64_t ld,
                                          ants_out rec, double* d_coef, int64_t* d_counts,
                                          void* hip_stream) {
  if (!set || !cfg || !d_coef) return set_error(ANTS_E_ARG, "ants_fit_axial_lrf: NULL argument");
  if (cfg->nb < 4 || cfg->nb > kFitMaxCoef - 2)
    return set_error(ANTS_E_ARG, "ants_fit_axial_lrf: nb = %d outside 4..%d", cfg->nb,
                     kFitMaxCoef - 2);
  if (!(cfg->lo >= 0.0 && cfg->hi > cfg->lo && cfg->hi < 1e300))
    return set_error(ANTS_E_ARG, "ants_fit_axial_lrf: domain [%g, %g] invalid", cfg->lo, cfg->hi);
  if (!(cfg->ridge >= 0.0 && cfg->ridge < 1e300))
    return set_error(ANTS_E_ARG, "ants_fit_axial_lrf: ridge %g invalid", cfg->ridge);
  if (n_events < 0) return set_error(ANTS_E_ARG, "ants_fit_axial_lrf: n_events < 0");
  if (n_events > 0 && (!d_signals || !rec_ok(rec)))
    return set_error(ANTS_E_ARG, "ants_fit_axial_lrf: NULL signals or reconstruction field");
  if (ld < set->ns) return set_error(ANTS_E_ARG, "ants_fit_axial_lrf: ld < n_sensors");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || set->device != dev)
    return set_error(ANTS_E_ARG, "ants_fit_axial_lrf: set on another device");
  hipStream_t s = (hipStream_t)hip_stream;
  const int nc = cfg->nb + 2;
  const int stride = nc * 5 + 2;
  int64_t blocks = (n_events + kFitWaves - 1) / kFitWaves;
  const int64_t cap = (int64_t)num_cu() * 8;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  const int nwaves = (int)blocks * kFitWaves;
  hipError_t e = ensure(&set->ws_fit, &set->ws_fit_bytes,
                        ((size_t)nwaves + 1) * stride * sizeof(double));
  if (e != hipSuccess) return hip_error(e, "ants_fit_axial_lrf workspace");
  FitP P;
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
  P.E = rec.E;
  P.chi2 = rec.chi2;
  P.ndf = rec.ndf;
  P.status = rec.status;
  P.chi2ndf_max = cfg->chi2ndf_max;
  P.nb = cfg->nb;
  P.nc = nc;
  P.lo = cfg->lo;
  P.hi = cfg->hi;
  P.inv_d = (double)(cfg->nb - 1) / (cfg->hi - cfg->lo);
  P.part = (double*)set->ws_fit;
  P.stride = stride;
  const size_t smem = (size_t)kFitWaves * kFitCopies * nc * 5 * sizeof(double);
  hipLaunchKernelGGL(fit_accum_kernel, dim3((unsigned)blocks), dim3(64 * kFitWaves), smem, s, P);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "ants_fit_axial_lrf accumulation");
  SolveP S;
  S.part = P.part;
  S.stride = stride;
  S.nwaves = nwaves;
  S.nc = nc;
  S.ridge = cfg->ridge;
  S.sums = P.part + (size_t)nwaves * stride;
  S.coef = d_coef;
  S.counts = d_counts;
  hipLaunchKernelGGL(fit_reduce_kernel, dim3(stride), dim3(256), 0, s, S);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, "ants_fit_axial_lrf reduction");
  hipLaunchKernelGGL(fit_solve_kernel, dim3(1), dim3(64), 0, s, S);
  e = hipGetLastError();
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_fit_axial_lrf solve");
}
