// Flood-field event generator on the device: events drawn from the LRF
// model itself (positions uniform over a disc or square and in depth,
// energies uniform, Sec. 4.1.1 "flood field"), expected counts
// mu_i = A g_i L_i with sum_active mu_i = E_tot, and Poisson counts.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC'11), keyed by the 64-bit seed,
// counter = (event index, stream, call).  Poisson draws: inversion by
// sequential search below a mean of 10, and above it the transformed
// rejection method with squeeze of W. Hoermann, "The transformed rejection
// method for generating Poisson random variables" (1993).
//
// One wavefront per event, lanes = active sensors.
#include <math.h>

#include "ants_internal.h"
#include "lrf64.h"

namespace ants {
namespace {

struct U4 {
  uint32_t v[4];
};

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += W0;
    k1 += W1;
  }
  U4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// (0,1) double from two 32-bit words: the top 53 bits, centred in their cell
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  uint64_t k = (((uint64_t)a << 32) | b) >> 11;
  return ((double)k + 0.5) * 0x1.0p-53;
}

__device__ double poisson_draw(double mu, uint32_t g0, uint32_t g1, uint32_t stream,
                               uint32_t k0, uint32_t k1) {
  if (!(mu > 0.0)) return 0.0;
  if (mu < 10.0) {
    U4 w = philox4x32_10(g0, g1, stream, 0u, k0, k1);
    double u = u53(w.v[0], w.v[1]);
    double p = exp(-mu), s = p;
    int k = 0;
    while (u > s && k < 1000) {
      ++k;
      p *= mu / k;
      s += p;
    }
    return (double)k;
  }
  const double slam = sqrt(mu), loglam = log(mu);
  const double b = 0.931 + 2.53 * slam;
  const double a = -0.059 + 0.02483 * b;
  const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
  const double vr = 0.9277 - 3.6224 / (b - 2.0);
  for (uint32_t t = 0; t < 64; ++t) {
    U4 w = philox4x32_10(g0, g1, stream, t, k0, k1);
    double U = u53(w.v[0], w.v[1]) - 0.5;
    double V = u53(w.v[2], w.v[3]);
    double us = 0.5 - fabs(U);
    double k = floor((2.0 * a / us + b) * U + mu + 0.43);
    if (us >= 0.07 && V <= vr) return k;
    if (k < 0.0 || (us < 0.013 && V > us)) continue;
    if (log(V) + log(invalpha) - log(a / (us * us) + b) <= -mu + k * loglam - lgamma(k + 1.0))
      return k;
  }
  return floor(mu + 0.5);
}

template <int KIND>
__global__ void __launch_bounds__(256)
gen_kernel(DevLrf L, GenP P, int64_t waves_total) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t e = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv; e < P.n; e += waves_total) {
    const uint64_t gidx = P.first + (uint64_t)e;
    const uint32_t g0 = (uint32_t)gidx, g1 = (uint32_t)(gidx >> 32);
    U4 wa = philox4x32_10(g0, g1, 0xFFFFFFFFu, 0u, P.k0, P.k1);
    U4 wb = philox4x32_10(g0, g1, 0xFFFFFFFFu, 1u, P.k0, P.k1);
    double u1 = u53(wa.v[0], wa.v[1]), u2 = u53(wa.v[2], wa.v[3]);
    double u3 = u53(wb.v[0], wb.v[1]), u4 = u53(wb.v[2], wb.v[3]);
    double x, y;
    if (P.region == 0) {
      double r = P.extent * sqrt(u1), phi = 6.283185307179586 * u2;
      x = r * cos(phi);
      y = r * sin(phi);
    } else {
      x = -P.extent + 2.0 * P.extent * u1;
      y = -P.extent + 2.0 * P.extent * u2;
    }
    double z = P.z_hi > P.z_lo ? P.z_lo + (P.z_hi - P.z_lo) * u3 : P.z_lo;
    double E = P.e_lo + (P.e_hi - P.e_lo) * u4;

    float* row = P.sig + (int64_t)e * L.ns;
    for (int c = lane; c < L.ns; c += 64) row[c] = 0.f;
    double gl[kSlots];
    double S = 0.0;
#pragma unroll
    for (int q = 0; q < kSlots; ++q) {
      int a = lane + 64 * q;
      gl[q] = 0.0;
      if (a < L.na) {
        gl[q] = L.g[a] * lrf64<KIND>(L, a, x, y, z);
        S += gl[q];
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) S += __shfl_xor(S, o);
    double A = S > 0.0 ? E / S : 0.0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < kSlots; ++q) {
      int a = lane + 64 * q;
      if (a < L.na) {
        double mu = A * gl[q];
        double n = P.noiseless ? mu : poisson_draw(mu, g0, g1, (uint32_t)L.col[a], P.k0, P.k1);
        row[L.col[a]] = (float)n;
      }
    }
    if (P.truth && lane < 4) {
      double v = lane == 0 ? x : lane == 1 ? y : lane == 2 ? z : E;
      P.truth[(int64_t)e * 4 + lane] = (float)v;
    }
  }
}

}  // namespace

hipError_t launch_gen(const DevLrf& L, const GenP& P, hipStream_t stream, int max_blocks) {
  int64_t blocks = (P.n + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  int64_t waves_total = blocks * kWavesPerBlock;
  dim3 g((unsigned)blocks), b(64 * kWavesPerBlock);
  if (L.kind == ANTS_LRF_AXIAL)
    hipLaunchKernelGGL(gen_kernel<ANTS_LRF_AXIAL>, g, b, 0, stream, L, P, waves_total);
  else if (L.kind == ANTS_LRF_XY)
    hipLaunchKernelGGL(gen_kernel<ANTS_LRF_XY>, g, b, 0, stream, L, P, waves_total);
  else if (L.kind == ANTS_LRF_COMPOSITE)
    hipLaunchKernelGGL(gen_kernel<ANTS_LRF_COMPOSITE>, g, b, 0, stream, L, P, waves_total);
  else if (L.kind == ANTS_LRF_SLICED)
    hipLaunchKernelGGL(gen_kernel<ANTS_LRF_SLICED>, g, b, 0, stream, L, P, waves_total);
  else
    hipLaunchKernelGGL(gen_kernel<ANTS_LRF_RZ>, g, b, 0, stream, L, P, waves_total);
  return hipGetLastError();
}

}  // namespace ants
