// k-NN reconstruction (Sec. 5.1.4): an event is the point of its
// normalised active-sensor signals n_i / N; its position is the mean of the
// known positions of the k calibration events closest to it (squared
// Euclidean distance), the lower calibration index first on equal
// distances.
//
// Exact brute force: the distance decides which events are neighbours, so
// it is computed in single precision in a fixed order (sensor order, each
// subtraction, square and sum rounded as written; rows padded with zeros,
// which add exactly nothing) and every pair is examined.  One thread per
// query holds its normalised signals and its sorted k best in registers;
// a block streams the calibration rows through LDS in tiles that all its
// threads read by broadcast.
#include <math.h>

#include "ants_internal.h"

namespace ants {
namespace {

constexpr int kKnnThreads = 256;
constexpr int kKnnLdsBytes = 32768;

// padded row width for na active sensors (rows of 4-float groups)
int knn_pad(int na) { return na <= 24 ? 24 : na <= 40 ? 40 : na <= 64 ? 64 : 128; }

struct KnnNormP {
  const float* sig;     // [m][ns]
  int64_t ns, m;
  const int32_t* col;   // [na] signal column of each active sensor
  int na, nap;
  float* cal;           // [m][nap]
};

// normalised signals of one row in double then single precision; invalid
// rows (N <= 0, or a non-finite or negative active signal) get +inf in
// column 0, so their distance is +inf and they never become neighbours.
// Returns the status bits.
__device__ __forceinline__ int knn_norm_row(const float* row, const int32_t* col, int na, int nap,
                                            float* out) {
  bool bad = false;
  double N = 0.0;
  for (int a = 0; a < na; ++a) {
    const float n = row[col[a]];
    if (!(n >= 0.f) || !(n < __builtin_huge_valf())) bad = true;
    else N += (double)n;
  }
  const int st = na == 0 ? ANTS_EV_NO_ACTIVE : bad ? ANTS_EV_BAD_INPUT
                 : !(N > 0.0) ? ANTS_EV_EMPTY : 0;
  for (int a = 0; a < nap; ++a) out[a] = 0.f;
  if (st) {
    out[0] = __builtin_huge_valf();
    return st;
  }
  for (int a = 0; a < na; ++a) out[a] = (float)((double)row[col[a]] / N);
  return 0;
}

__global__ void knn_norm_kernel(KnnNormP P) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < P.m) knn_norm_row(P.sig + c * P.ns, P.col, P.na, P.nap, P.cal + c * P.nap);
}

struct KnnP {
  const float* cal;     // [m][nap]
  const float* pos;     // [m][3]
  int64_t m;
  int k;
  const float* sig;     // queries [n][ns]
  int64_t ns, n;
  const int32_t* col;
  int na;
  float* xyz;           // [n][3]
  int32_t* status;      // [n]
  int32_t* idx;         // [n][k] or NULL
  float* dist;          // [n][k] or NULL
};

template <int NAP, int KMAX>
__global__ void __launch_bounds__(kKnnThreads) knn_kernel(KnnP P) {
#pragma clang fp contract(off)
  constexpr int T = kKnnLdsBytes / (4 * NAP);   // calibration rows per tile
  __shared__ float4 tile[T * NAP / 4];
  const int64_t e = (int64_t)blockIdx.x * kKnnThreads + threadIdx.x;
  const bool live = e < P.n;
  // normalised query in registers (the same steps as knn_norm_row, with
  // compile-time indices)
  float q[NAP];
  int st = ANTS_EV_EMPTY;
  {
    const float* row = P.sig + (live ? e : 0) * P.ns;
    bool bad = false;
    double N = 0.0;
#pragma unroll
    for (int a = 0; a < NAP; ++a) {
      q[a] = 0.f;
      if (live && a < P.na) {
        q[a] = row[P.col[a]];
        if (!(q[a] >= 0.f) || !(q[a] < __builtin_huge_valf())) bad = true;
        else N += (double)q[a];
      }
    }
    st = P.na == 0 ? ANTS_EV_NO_ACTIVE : bad ? ANTS_EV_BAD_INPUT : !(N > 0.0) ? ANTS_EV_EMPTY : 0;
#pragma unroll
    for (int a = 0; a < NAP; ++a) q[a] = (st == 0 && a < P.na) ? (float)((double)q[a] / N) : 0.f;
  }
  // an invalid query compares as +inf everywhere and keeps an empty list
  const bool search = live && st == 0;
  float bd[KMAX];
  int bi[KMAX];
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    bd[j] = __builtin_huge_valf();
    bi[j] = -1;
  }
  const int k = P.k;
  for (int64_t c0 = 0; c0 < P.m; c0 += T) {
    const int nt = (int)(P.m - c0 < T ? P.m - c0 : T);
    __syncthreads();
    const float4* src = (const float4*)(P.cal + c0 * NAP);
    for (int i = threadIdx.x; i < nt * NAP / 4; i += kKnnThreads) tile[i] = src[i];
    __syncthreads();
    if (!search) continue;
    for (int t = 0; t < nt; ++t) {
      const float4* row = tile + t * (NAP / 4);
      float s = 0.f;
#pragma unroll
      for (int a4 = 0; a4 < NAP / 4; ++a4) {
        const float4 c = row[a4];
        float d = q[4 * a4] - c.x;
        s = s + d * d;
        d = q[4 * a4 + 1] - c.y;
        s = s + d * d;
        d = q[4 * a4 + 2] - c.z;
        s = s + d * d;
        d = q[4 * a4 + 3] - c.w;
        s = s + d * d;
      }
      // rows come in increasing index, so an equal distance never displaces
      // an earlier neighbour; insert after the entries not above s
      if (s < bd[k - 1]) {
        const int ci = (int)(c0 + t);
#pragma unroll
        for (int j = KMAX - 1; j >= 0; --j) {
          if (j < k) {
            const float prev = j > 0 ? bd[j - 1] : -__builtin_huge_valf();
            if (prev > s) {
              bd[j] = bd[j - 1];
              bi[j] = bi[j - 1];
            } else if (bd[j] > s) {
              bd[j] = s;
              bi[j] = ci;
            }
          }
        }
      }
    }
  }
  if (!live) return;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  int kk = 0;
#pragma unroll
  for (int j = 0; j < KMAX; ++j) {
    if (j < k && bi[j] >= 0) {
      sx += (double)P.pos[3 * (int64_t)bi[j]];
      sy += (double)P.pos[3 * (int64_t)bi[j] + 1];
      sz += (double)P.pos[3 * (int64_t)bi[j] + 2];
      ++kk;
    }
    if (j < k && P.idx) P.idx[e * k + j] = bi[j];
    if (j < k && P.dist) P.dist[e * k + j] = bd[j];
  }
  if (st == 0 && kk == 0) st = ANTS_EV_NO_VALID_NODE;
  const float nan = __builtin_nanf("");
  P.xyz[3 * e] = kk ? (float)(sx / (double)kk) : nan;
  P.xyz[3 * e + 1] = kk ? (float)(sy / (double)kk) : nan;
  P.xyz[3 * e + 2] = kk ? (float)(sz / (double)kk) : nan;
  P.status[e] = st;
}

template <int NAP>
hipError_t launch_knn_n(const KnnP& P, hipStream_t s) {
  const dim3 grid((unsigned)((P.n + kKnnThreads - 1) / kKnnThreads));
  if (P.k <= 8) hipLaunchKernelGGL((knn_kernel<NAP, 8>), grid, dim3(kKnnThreads), 0, s, P);
  else if (P.k <= 16) hipLaunchKernelGGL((knn_kernel<NAP, 16>), grid, dim3(kKnnThreads), 0, s, P);
  else hipLaunchKernelGGL((knn_kernel<NAP, 32>), grid, dim3(kKnnThreads), 0, s, P);
  return hipGetLastError();
}

}  // namespace
}  // namespace ants

using namespace ants;

struct ants_knn {
  int device = 0;
  int ns = 0, na = 0, nap = 0;
  int64_t m = 0;
  int32_t* col = nullptr;
  float* cal = nullptr;
  float* pos = nullptr;
};

extern "C" {

ants_status ants_knn_create(ants_lrfset* set, int64_t n_cal, const float* d_signals,
                            const float* d_pos, ants_knn** out, void* hip_stream) {
  if (!out) return set_error(ANTS_E_ARG, "ants_knn_create: NULL out");
  *out = nullptr;
  if (!set || !d_signals || !d_pos)
    return set_error(ANTS_E_ARG, "ants_knn_create: NULL set, signals or positions");
  if (n_cal < 1 || n_cal > ((int64_t)1 << 31) - 1)
    return set_error(ANTS_E_ARG, "n_cal = %lld out of range", (long long)n_cal);
  if (set->d.na > 128)
    return set_error(ANTS_E_UNSUPPORTED, "k-NN supports at most 128 active sensors (%d)",
                     set->d.na);
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != set->device) return set_error(ANTS_E_ARG, "LRF set lives on another device");
  ants_knn* K = new ants_knn();
  K->device = dev;
  K->ns = set->ns;
  K->na = set->d.na;
  K->nap = knn_pad(K->na);
  K->m = n_cal;
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = hipMalloc((void**)&K->cal, (size_t)n_cal * K->nap * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&K->pos, (size_t)n_cal * 3 * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void**)&K->col, (size_t)(K->na > 0 ? K->na : 1) * 4);
  if (e == hipSuccess && K->na > 0)
    e = hipMemcpyAsync(K->col, set->d.col, (size_t)K->na * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(K->pos, d_pos, (size_t)n_cal * 3 * sizeof(float), hipMemcpyDeviceToDevice,
                       s);
  if (e == hipSuccess) {
    KnnNormP P{d_signals, K->ns, n_cal, K->col, K->na, K->nap, K->cal};
    hipLaunchKernelGGL(knn_norm_kernel, dim3((unsigned)((n_cal + 255) / 256)), dim3(256), 0, s, P);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    ants_knn_destroy(K);
    return hip_error(e, "ants_knn_create");
  }
  *out = K;
  return ANTS_OK;
}

ants_status ants_knn_destroy(ants_knn* K) {
  if (!K) return ANTS_OK;
  if (K->cal) (void)hipFree(K->cal);
  if (K->pos) (void)hipFree(K->pos);
  if (K->col) (void)hipFree(K->col);
  delete K;
  return ANTS_OK;
}

ants_status ants_knn_reconstruct(ants_knn* K, int32_t k, int64_t n_events,
                                 const float* d_signals, float* d_xyz, int32_t* d_status,
                                 int32_t* d_idx, float* d_dist, void* hip_stream) {
  if (!K) return set_error(ANTS_E_ARG, "ants_knn_reconstruct: NULL handle");
  if (k < 1 || k > 32) return set_error(ANTS_E_ARG, "k = %d outside 1..32", k);
  if (n_events < 0 || n_events > ((int64_t)1 << 31) - 1)
    return set_error(ANTS_E_ARG, "n_events = %lld out of range", (long long)n_events);
  if (n_events == 0) return ANTS_OK;
  if (!d_signals || !d_xyz || !d_status)
    return set_error(ANTS_E_ARG, "NULL signal, position or status pointer");
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != K->device) return set_error(ANTS_E_ARG, "k-NN set lives on another device");
  KnnP P{K->cal, K->pos, K->m, k, d_signals, K->ns, n_events, K->col, K->na,
         d_xyz, d_status, d_idx, d_dist};
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = K->nap == 24 ? launch_knn_n<24>(P, s)
                 : K->nap == 40 ? launch_knn_n<40>(P, s)
                 : K->nap == 64 ? launch_knn_n<64>(P, s)
                                : launch_knn_n<128>(P, s);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_knn_reconstruct launch");
}

}  // extern "C"
