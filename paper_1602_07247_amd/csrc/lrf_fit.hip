// LRF fit from events (the LRF module computing LRFs from signals and event
// positions, Sec. 6; sensors in groups sharing one LRF with relative gains,
// Sec. 6.2; gains re-calculated within fixed groups, Sec. 6.3; alternated
// with the reconstruction by the iterative procedure, Sec. 8).
//
// Axial LRF, one cubic B-spline table of nc = nb + 2 coefficients per group:
// least squares on the estimates n / (E g) of L(r), one per (event, member
// sensor) pair inside the domain.  The normal matrix is banded (a pair
// touches four consecutive coefficients), so each wave accumulates its band
// (4 diagonals) and right-hand side in FP64 in its own LDS area; a group's
// waves' partial sums are added by a fixed tree and one wave per group
// solves its system by Cholesky.  Results do not depend on the launch's
// timing.
#include <math.h>
#include <string.h>

#include "ants_internal.h"
#include "lrf64.h"

using namespace ants;

namespace {

constexpr int kFitMaxCoef = 64;
constexpr int kFitWaves = 4;   // waves per block of the accumulation
constexpr int kFitCopies = 4;  // accumulator copies per wave (lane % 4), fewer same-address atomics
constexpr int kFitMaxGroups = 4096;

struct FitP {
  const int32_t* col;
  const double *X, *Y, *g;
  int na;
  const float* sig;
  int64_t ld, n;
  const float *x, *y, *E, *chi2;
  const int32_t *ndf, *status;
  const float* shift;   // [n][2] added to (x, y), or NULL
  double chi2ndf_max;
  int nb, nc;
  double lo, hi, inv_d;
  // groups: members (compact sensor indices) of group g are
  // members[moff[g] .. moff[g + 1]); blocks g * chunks .. (g + 1) * chunks - 1
  const int32_t *members, *moff;
  int chunks;
  // gain mode: the fixed table of each group (tables + g * nc); per wave
  // three sums per member (sum t L, sum L^2, pairs) instead of normal
  // equations
  const double* tables;
  int acc_n;         // accumulated values per copy: nc * 5 (fit) or 3 * max members (gains)
  double* part;      // [groups * waves per group][stride]: sums, then events and pairs
  int stride;
};

// Member lists of the groups from a per-sensor group array (by sensor id;
// entries outside [0, groups) leave the sensor out), in increasing compact
// index: one thread, a few hundred sensors.
__global__ void fit_groups_kernel(const int32_t* group, const int32_t* col, int na, int groups,
                                  int32_t* moff, int32_t* members) {
  if (threadIdx.x != 0) return;
  auto gof = [&](int a) { return group ? group[col[a]] : 0; };   // NULL: one group
  for (int g = 0; g <= groups; ++g) moff[g] = 0;
  for (int a = 0; a < na; ++a) {
    const int g = gof(a);
    if (g >= 0 && g < groups) moff[g + 1] += 1;
  }
  for (int g = 0; g < groups; ++g) moff[g + 1] += moff[g];
  for (int g = 0; g < groups; ++g) {
    int k = moff[g];
    for (int a = 0; a < na; ++a)
      if (gof(a) == g) members[k++] = a;
  }
}

// One block per (group, chunk of events), waves over events.  Groups of at
// least 32 members: one event per wave at a time, lanes over members;
// smaller groups: 64 / members events per wave, lanes over (event,
// member).  Pairs are added into the wave's LDS area (kFitCopies copies,
// lane % kFitCopies) with FP64 atomics; the area goes to the partials.
template <bool GAINS>
__global__ void __launch_bounds__(64 * kFitWaves) fit_accum_kernel(FitP P) {
  extern __shared__ double fsm[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nc = P.nc, an = P.acc_n;
  const int grp = blockIdx.x / P.chunks, chunk = blockIdx.x - grp * P.chunks;
  const int32_t* mem = P.members + P.moff[grp];
  const int nm = P.moff[grp + 1] - P.moff[grp];
  const double* tab = GAINS ? P.tables + (int64_t)grp * nc : nullptr;
  double* wacc = fsm + wv * (an * kFitCopies);
  double* acc = wacc + (lane % kFitCopies) * an;
  for (int i = lane; i < an * kFitCopies; i += 64) wacc[i] = 0.0;
  __syncthreads();
  const int64_t gw = (int64_t)chunk * kFitWaves + wv;        // wave within the group
  const int64_t nw = (int64_t)P.chunks * kFitWaves;          // waves of the group
  // lane -> (event slot, first member); members in steps of mstep
  const int epw = (nm >= 32 || nm == 0) ? 1 : 64 / nm;
  const int slot = epw == 1 ? 0 : lane / nm;
  const int m0 = epw == 1 ? lane : lane - slot * nm;
  const int mstep = epw == 1 ? 64 : nm;
  const bool live = slot < epw;
  double used = 0.0, pairs = 0.0;
  for (int64_t k0 = 0; gw + k0 * nw < P.n; k0 += epw) {
    const int64_t e = gw + (k0 + slot) * nw;
    if (!live || e >= P.n) continue;
    const float Ef = P.E[e];
    bool ok = (P.status[e] & kEvFailed) == 0 && Ef > 0.f && Ef < __builtin_huge_valf();
    if (P.chi2ndf_max > 0.0) {
      const int d = P.ndf[e];
      ok = ok && d > 0 && (double)P.chi2[e] / (double)d <= P.chi2ndf_max;
    }
    if (!ok) continue;
    if (m0 == 0) used += 1.0;
    double xe = P.x[e], ye = P.y[e];
    if (P.shift) {
      xe += (double)P.shift[2 * e];
      ye += (double)P.shift[2 * e + 1];
    }
    const double Ee = Ef;
    const float* row = P.sig + e * P.ld;
    for (int mi = m0; mi < nm; mi += mstep) {
      const int a = mem[mi];
      const double dx = xe - P.X[a], dy = ye - P.Y[a];
      const double r = sqrt(dx * dx + dy * dy);
      int m;
      double t;
      if (!locate64(r, P.nb, P.lo, P.hi, P.inv_d, m, t)) continue;
      double b[4];
      bweights64(t, b);
      if constexpr (GAINS) {
        // the reconstruction's LRF of the group (clamped at 0) and the
        // sensor's estimate n / E of g L
        double Lv = tab[m] * b[0] + tab[m + 1] * b[1] + tab[m + 2] * b[2] + tab[m + 3] * b[3];
        Lv = Lv > 0.0 ? Lv : 0.0;
        const double te = (double)row[P.col[a]] / Ee;
        atomicAdd(&acc[3 * mi], te * Lv);
        atomicAdd(&acc[3 * mi + 1], Lv * Lv);
        atomicAdd(&acc[3 * mi + 2], 1.0);
      } else {
        const double tg = (double)row[P.col[a]] / (Ee * P.g[a]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          atomicAdd(&acc[4 * nc + m + k], b[k] * tg);
#pragma unroll
          for (int l = k; l < 4; ++l) atomicAdd(&acc[4 * (m + k) + (l - k)], b[k] * b[l]);
        }
      }
      pairs += 1.0;
    }
  }
  __syncthreads();
  double* out = P.part + ((int64_t)grp * nw + gw) * P.stride;
  for (int i = lane; i < an; i += 64) {
    double v = wacc[i];
    for (int c = 1; c < kFitCopies; ++c) v += wacc[c * an + i];
    out[i] = v;
  }
  // events and pairs of the wave (each lane counted its own)
  for (int o = 32; o >= 1; o >>= 1) {
    used += __shfl_xor(used, o);
    pairs += __shfl_xor(pairs, o);
  }
  if (lane == 0) {
    out[an] = used;
    out[an + 1] = pairs;
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
  int stride, nwaves, nc;   // nwaves: per group
  double ridge;
  double* sums;      // [groups][stride]: each group's wave partials added up
  double* coef;      // [groups][nc]
  int64_t* counts;   // [groups][2] or NULL
  // gains: members as in FitP, sensor columns, outputs per sensor column
  const int32_t *members, *moff, *col;
  double* gains;
  int64_t* gpairs;
};

// One block per (entry of the partials, group): the group's wave values
// added by a fixed tree (thread t takes waves t, t + 256, ...; then
// pairwise halving).
__global__ void __launch_bounds__(256) fit_reduce_kernel(SolveP P) {
  __shared__ double red[256];
  const int i = blockIdx.x, g = blockIdx.y, tid = threadIdx.x;
  const double* part = P.part + (int64_t)g * P.nwaves * P.stride;
  double s = 0.0;
  for (int w = tid; w < P.nwaves; w += 256) s += part[(int64_t)w * P.stride + i];
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) P.sums[(int64_t)g * P.stride + i] = red[0];
}

// gains within fixed tables: g = sum t L / sum L^2 per member (NaN without
// pairs or with sum L^2 = 0)
__global__ void fit_gains_finish_kernel(SolveP P, int groups) {
  const int g = blockIdx.x;
  if (g >= groups) return;
  const double* sm = P.sums + (int64_t)g * P.stride;
  for (int mi = threadIdx.x; mi < P.moff[g + 1] - P.moff[g]; mi += blockDim.x) {
    const int c = P.col[P.members[P.moff[g] + mi]];
    const double tl = sm[3 * mi], ll = sm[3 * mi + 1], np = sm[3 * mi + 2];
    P.gains[c] = (np > 0.0 && ll > 0.0) ? tl / ll : __builtin_nan("");
    if (P.gpairs) P.gpairs[c] = (int64_t)np;
  }
}

__global__ void __launch_bounds__(64) fit_solve_kernel(SolveP P) {
  __shared__ double band[kFitMaxCoef * 5 + 2];
  __shared__ double A[kFitMaxCoef][kFitMaxCoef + 1];
  __shared__ double y[kFitMaxCoef];
  const int lane = threadIdx.x, nc = P.nc, g = blockIdx.x;
  for (int i = lane; i < nc * 5 + 2; i += 64) band[i] = P.sums[(int64_t)g * P.stride + i];
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
    for (int i = 0; i < nc; ++i) P.coef[(int64_t)g * nc + i] = y[i];
    if (P.counts) {
      P.counts[2 * g] = (int64_t)band[nc * 5];
      P.counts[2 * g + 1] = (int64_t)band[nc * 5 + 1];
    }
  }
}

bool rec_ok(const ants_out& o) { return o.x && o.y && o.E && o.chi2 && o.ndf && o.status; }


// The fits share one driver: member lists, accumulation per (group, chunk),
// fixed-tree sums per group, then the Cholesky solves or the gain ratios.
ants_status fit_run(ants_lrfset* set, const ants_fit_cfg* cfg, int groups, const int32_t* d_group,
                    const double* d_tables, int64_t n_events, const float* d_signals, int64_t ld,
                    const ants_out& rec, const float* d_shift, double* d_coef, int64_t* d_counts,
                    double* d_gains, int64_t* d_pairs, hipStream_t s, const char* who) {
  const bool gains = d_tables != nullptr;
  if (cfg->nb < 4 || cfg->nb > kFitMaxCoef - 2)
    return set_error(ANTS_E_ARG, "%s: nb = %d outside 4..%d", who, cfg->nb, kFitMaxCoef - 2);
  if (!(cfg->lo >= 0.0 && cfg->hi > cfg->lo && cfg->hi < 1e300))
    return set_error(ANTS_E_ARG, "%s: domain [%g, %g] invalid", who, cfg->lo, cfg->hi);
  if (!(cfg->ridge >= 0.0 && cfg->ridge < 1e300))
    return set_error(ANTS_E_ARG, "%s: ridge %g invalid", who, cfg->ridge);
  if (groups < 1 || groups > kFitMaxGroups)
    return set_error(ANTS_E_ARG, "%s: %d groups outside 1..%d", who, groups, kFitMaxGroups);
  if (n_events < 0) return set_error(ANTS_E_ARG, "%s: n_events < 0", who);
  if (n_events > 0 && (!d_signals || !rec_ok(rec)))
    return set_error(ANTS_E_ARG, "%s: NULL signals or reconstruction field", who);
  if (ld < set->ns) return set_error(ANTS_E_ARG, "%s: ld < n_sensors", who);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || set->device != dev)
    return set_error(ANTS_E_ARG, "%s: set on another device", who);
  const int na = set->d.na, nc = cfg->nb + 2;
  const int acc_n = gains ? 3 * (na > 0 ? na : 1) : nc * 5;
  const int stride = acc_n + 2;
  const int64_t cap = (int64_t)num_cu() * 8;
  int64_t chunks = (n_events + kFitWaves - 1) / kFitWaves;
  const int64_t per_group = cap / groups > 0 ? cap / groups : 1;
  if (chunks > per_group) chunks = per_group;
  if (chunks < 1) chunks = 1;
  const int nw = (int)chunks * kFitWaves;
  // workspace: member lists (ints), then partials and group sums (doubles)
  const size_t ibytes = ((size_t)(na + groups + 1) * sizeof(int32_t) + 15) / 16 * 16;
  const size_t dcount = ((size_t)groups * nw + groups) * stride;
  hipError_t e = ensure(&set->ws_fit, &set->ws_fit_bytes, ibytes + dcount * sizeof(double));
  if (e != hipSuccess) return hip_error(e, who);
  int32_t* members = (int32_t*)set->ws_fit;
  int32_t* moff = members + na;
  double* part = (double*)((char*)set->ws_fit + ibytes);
  hipLaunchKernelGGL(fit_groups_kernel, dim3(1), dim3(64), 0, s, d_group, set->d.col, na, groups,
                     moff, members);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, who);
  FitP P;
  memset(&P, 0, sizeof(P));
  P.col = set->d.col;
  P.X = set->d.X;
  P.Y = set->d.Y;
  P.g = set->d.g;
  P.na = na;
  P.sig = d_signals;
  P.ld = ld;
  P.n = n_events;
  P.x = rec.x;
  P.y = rec.y;
  P.E = rec.E;
  P.chi2 = rec.chi2;
  P.ndf = rec.ndf;
  P.status = rec.status;
  P.shift = d_shift;
  P.chi2ndf_max = cfg->chi2ndf_max;
  P.nb = cfg->nb;
  P.nc = nc;
  P.lo = cfg->lo;
  P.hi = cfg->hi;
  P.inv_d = (double)(cfg->nb - 1) / (cfg->hi - cfg->lo);
  P.members = members;
  P.moff = moff;
  P.chunks = (int)chunks;
  P.tables = d_tables;
  P.acc_n = acc_n;
  P.part = part;
  P.stride = stride;
  const size_t smem = (size_t)kFitWaves * kFitCopies * acc_n * sizeof(double);
  const void* kern = gains ? (const void*)fit_accum_kernel<true> : (const void*)fit_accum_kernel<false>;
  if (smem > 65536) {
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (e != hipSuccess) return hip_error(e, who);
  }
  const dim3 grid((unsigned)(chunks * groups));
  if (gains)
    hipLaunchKernelGGL(fit_accum_kernel<true>, grid, dim3(64 * kFitWaves), smem, s, P);
  else
    hipLaunchKernelGGL(fit_accum_kernel<false>, grid, dim3(64 * kFitWaves), smem, s, P);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, who);
  SolveP S;
  memset(&S, 0, sizeof(S));
  S.part = part;
  S.stride = stride;
  S.nwaves = nw;
  S.nc = nc;
  S.ridge = cfg->ridge;
  S.sums = part + (size_t)groups * nw * stride;
  S.coef = d_coef;
  S.counts = d_counts;
  S.members = members;
  S.moff = moff;
  S.col = set->d.col;
  S.gains = d_gains;
  S.gpairs = d_pairs;
  hipLaunchKernelGGL(fit_reduce_kernel, dim3(stride, groups), dim3(256), 0, s, S);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_error(e, who);
  if (gains)
    hipLaunchKernelGGL(fit_gains_finish_kernel, dim3(groups), dim3(64), 0, s, S, groups);
  else
    hipLaunchKernelGGL(fit_solve_kernel, dim3(groups), dim3(64), 0, s, S);
  e = hipGetLastError();
  return e == hipSuccess ? ANTS_OK : hip_error(e, who);
}

}  // namespace

extern "C" ants_status ants_fit_axial_lrf(ants_lrfset* set, const ants_fit_cfg* cfg,
                                          int64_t n_events, const float* d_signals, int64_t ld,
                                          ants_out rec, double* d_coef, int64_t* d_counts,
                                          void* hip_stream) {
  if (!set || !cfg || !d_coef) return set_error(ANTS_E_ARG, "ants_fit_axial_lrf: NULL argument");
  return fit_run(set, cfg, 1, nullptr, nullptr, n_events, d_signals, ld, rec, nullptr, d_coef,
                 d_counts, nullptr, nullptr, (hipStream_t)hip_stream, "ants_fit_axial_lrf");
}

extern "C" ants_status ants_fit_axial_lrf_grouped(ants_lrfset* set, const ants_fit_cfg* cfg,
                                                  int32_t n_groups, const int32_t* d_group,
                                                  int64_t n_events, const float* d_signals,
                                                  int64_t ld, ants_out rec, const float* d_shift,
                                                  double* d_coef, int64_t* d_counts,
                                                  void* hip_stream) {
  if (!set || !cfg || !d_coef || !d_group)
    return set_error(ANTS_E_ARG, "ants_fit_axial_lrf_grouped: NULL argument");
  return fit_run(set, cfg, n_groups, d_group, nullptr, n_events, d_signals, ld, rec, d_shift,
                 d_coef, d_counts, nullptr, nullptr, (hipStream_t)hip_stream,
                 "ants_fit_axial_lrf_grouped");
}

extern "C" ants_status ants_fit_axial_gains(ants_lrfset* set, const ants_fit_cfg* cfg,
                                            int32_t n_tables, const double* d_tables,
                                            const int32_t* d_table_of, int64_t n_events,
                                            const float* d_signals, int64_t ld, ants_out rec,
                                            const float* d_shift, double* d_gains,
                                            int64_t* d_pairs, void* hip_stream) {
  if (!set || !cfg || !d_tables || !d_table_of || !d_gains)
    return set_error(ANTS_E_ARG, "ants_fit_axial_gains: NULL argument");
  return fit_run(set, cfg, n_tables, d_table_of, d_tables, n_events, d_signals, ld, rec, d_shift,
                 nullptr, nullptr, d_gains, d_pairs, (hipStream_t)hip_stream,
                 "ants_fit_axial_gains");
}
