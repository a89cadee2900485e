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
// 3 (nb0 + 2) + 3 in that index; one wave per group adds the relative
// ridge and solves it by banded Cholesky.
//
// Accumulation.  A pair's contribution is 136 products of its 16 patch
// weights and 16 right-side terms, all at its patch origin (m0, m1).  The
// second argument (z for r-z, y for XY) belongs to the event, so every pair
// of an event has the same m1: blocks own one m1 row and one chunk of
// events, take the events of their row, and each wave sums its pairs into
// its own LDS copy of the row's per-origin sums (152 FP64 per origin and
// group).  The block adds its waves' copies in wave order, a second kernel
// adds the chunks in chunk order, and one wave per group adds the origins
// into the band in origin order: the same bits on every call.  When a
// row's sums for every group do not fit two waves' LDS (many groups), the
// pairs go straight to the band by FP64 global atomics instead (sums in
// arrival order: the last bits may differ from call to call).
#include <math.h>
#include <string.h>

#include <algorithm>

#include "ants_internal.h"
#include "lrf64.h"

using namespace ants;

namespace {

constexpr int kFit2MaxKnots = 64;
constexpr int kFit2MaxGroups = 1024;
constexpr int kFit2Terms = 152;     // 136 patch products (i <= j) + 16 right-side terms
constexpr int kFit2Stride = 153;    // per-origin stride in LDS (odd: spreads the banks)
constexpr int kFit2LdsBytes = 160 * 1024;

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
  const double* base;  // composite residual: axial spline subtracted at r, or NULL
  int base_nb;
  double base_lo, base_hi, base_inv;
  int zwin;            // 1: only events with zw_lo <= z < zw_hi
  double zw_lo, zw_hi;
  int rz;              // 1: arguments (r, z); 0: (x, y)
  int nb0, nb1, nc0, nc, bw;
  double lo0, hi0, lo1, hi1, inv_d0, inv_d1;
  const int32_t* group;   // per sensor index
  int groups;
  double* band;        // [groups][nc][bw + 1]: entry (i, i + k) at [i][k]
  double* rhs;         // [groups][nc]
  unsigned long long* pairs;   // [groups]
  unsigned long long* used;    // [1]
  // row accumulation: rows = nb1 - 1, no = nb0 - 1 origins per row
  int rows, no, chunks;
  int64_t chunk_len;
  double* part;        // [chunks][rows][groups * no * kFit2Terms]
};

// the composite's axial part at distance r: the spline, not clamped, 0
// outside its domain
__device__ __forceinline__ double base_value(const Fit2P& P, double r) {
  int m;
  double t;
  if (!locate64(r, P.base_nb, P.base_lo, P.base_hi, P.base_inv, m, t)) return 0.0;
  double b[4];
  bweights64(t, b);
  const double* c = P.base + m;
  return b[0] * c[0] + b[1] * c[1] + b[2] * c[2] + b[3] * c[3];
}

// the event's filter (status failure bits, energy, chi2/ndf)
__device__ __forceinline__ bool fit2_keep(const Fit2P& P, int64_t e) {
  const float Ef = P.E[e];
  bool ok = (P.status[e] & kEvFailed) == 0 && Ef > 0.f && Ef < __builtin_huge_valf();
  if (P.chi2ndf_max > 0.0) {
    const int d = P.ndf[e];
    ok = ok && d > 0 && (double)P.chi2[e] / (double)d <= P.chi2ndf_max;
  }
  if (P.zwin) {
    const double z = P.z[e];
    ok = ok && z >= P.zw_lo && z < P.zw_hi;
  }
  return ok;
}

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
    if (!fit2_keep(P, e)) continue;   // uniform over the wave
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
      double tg = (double)row[P.col[a]] / (Ee * P.g[a]);
      if (P.base) {
        const double dx = xe - P.X[a], dy = ye - P.Y[a];
        tg -= base_value(P, sqrt(dx * dx + dy * dy));
      }
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

// Row accumulation (see the file comment).  Block (row, chunk); each wave
// takes 64-event tiles of the chunk in turn, picks the events of its row
// and adds their pairs (lanes over sensors, slot q holding sensor
// lane + 64 q) into its LDS copy acc[(group * no + m0) * kFit2Stride + term];
// after the waves' copies come the block's pair counters, one per group.
// The signals of up to four picked events are loaded before any of them is
// summed, so their memory latency overlaps.
__global__ void __launch_bounds__(256) fit2_rows_kernel(Fit2P P) {
  constexpr int Q = kMaxSensors / 64;
  constexpr int B = 4;
  extern __shared__ double f2s[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int row = blockIdx.x % P.rows, chunk = blockIdx.x / P.rows;
  const int per = P.groups * P.no * kFit2Stride;
  double* acc = f2s + (int64_t)wave * per;
  unsigned long long* cnt = (unsigned long long*)(f2s + (int64_t)nwv * per);
  for (int i = lane; i < per; i += 64) acc[i] = 0.0;
  for (int i = threadIdx.x; i < P.groups; i += blockDim.x) cnt[i] = 0ull;
  int scol[Q], sgr[Q];
  double sX[Q], sY[Q], sg[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int a = lane + 64 * q;
    scol[q] = 0;
    sgr[q] = -1;
    sX[q] = sY[q] = 0.0;
    sg[q] = 1.0;
    if (a < P.na) {
      scol[q] = P.col[a];
      const int gr = P.group[scol[q]];
      sgr[q] = (gr >= 0 && gr < P.groups) ? gr : -1;
      sX[q] = P.X[a];
      sY[q] = P.Y[a];
      sg[q] = P.g[a];
    }
  }
  __syncthreads();
  const int64_t e0 = (int64_t)chunk * P.chunk_len;
  const int64_t e1 = e0 + P.chunk_len < P.n ? e0 + P.chunk_len : P.n;
  for (int64_t base = e0 + 64 * wave; base < e1; base += 64 * nwv) {
    const int64_t e = base + lane;
    bool take = false, ok = false;
    int m1 = 0;
    double t1 = 0.0;
    if (e < e1) {
      ok = fit2_keep(P, e);
      double w = P.rz ? (double)P.z[e] : (double)P.y[e];
      if (!P.rz && P.shift) w += (double)P.shift[2 * e + 1];
      take = ok && locate64(w, P.nb1, P.lo1, P.hi1, P.inv_d1, m1, t1) && m1 == row;
    }
    if (row == 0) {   // every kept event once, from its chunk's row-0 block
      const uint64_t okm = __ballot(ok);
      if (lane == 0 && okm) atomicAdd(P.used, (unsigned long long)__popcll(okm));
    }
    uint64_t m = __ballot(take);
    while (m) {
      int lv[B];
#pragma unroll
      for (int c = 0; c < B; ++c) {
        lv[c] = m ? __builtin_ctzll(m) : -1;
        m &= m - 1;
      }
      float sv[B][Q];
      double xe[B], ye[B], Ee[B], te[B];
#pragma unroll
      for (int c = 0; c < B; ++c) {
        xe[c] = ye[c] = te[c] = 0.0;
        Ee[c] = 1.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) sv[c][q] = 0.f;
        if (lv[c] < 0) continue;   // uniform
        const int64_t ev = base + lv[c];
        te[c] = __shfl(t1, lv[c]);
        xe[c] = P.x[ev];
        ye[c] = P.y[ev];
        if (P.shift) {
          xe[c] += (double)P.shift[2 * ev];
          ye[c] += (double)P.shift[2 * ev + 1];
        }
        Ee[c] = P.E[ev];
        const float* srow = P.sig + ev * P.ld;
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (sgr[q] >= 0) sv[c][q] = srow[scol[q]];
      }
#pragma unroll
      for (int c = 0; c < B; ++c) {
        if (lv[c] < 0) continue;   // uniform
        double b1[4];
        bweights64(te[c], b1);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          if (sgr[q] < 0) continue;
          double u;
          if (P.rz) {
            const double dx = xe[c] - sX[q], dy = ye[c] - sY[q];
            u = sqrt(dx * dx + dy * dy);
          } else {
            u = xe[c];
          }
          int m0;
          double t0;
          if (!locate64(u, P.nb0, P.lo0, P.hi0, P.inv_d0, m0, t0)) continue;
          double b0[4];
          bweights64(t0, b0);
          double tg = (double)sv[c][q] / (Ee[c] * sg[q]);
          if (P.base) {
            const double dx = xe[c] - sX[q], dy = ye[c] - sY[q];
            tg -= base_value(P, sqrt(dx * dx + dy * dy));
          }
          double wt[16];
#pragma unroll
          for (int qq = 0; qq < 4; ++qq)
#pragma unroll
            for (int p = 0; p < 4; ++p) wt[4 * qq + p] = b1[qq] * b0[p];
          double* o = acc + (sgr[q] * P.no + m0) * kFit2Stride;
          int k = 0;
#pragma unroll
          for (int i = 0; i < 16; ++i)
#pragma unroll
            for (int jj = i; jj < 16; ++jj) atomicAdd(&o[k++], wt[i] * wt[jj]);
#pragma unroll
          for (int i = 0; i < 16; ++i) atomicAdd(&o[136 + i], wt[i] * tg);
          atomicAdd(&cnt[sgr[q]], 1ull);
        }
      }
    }
  }
  __syncthreads();
  // the block's sum over its waves, in wave order, to its chunk's slot
  const int terms = P.groups * P.no * kFit2Terms;
  double* dst = P.part + ((int64_t)chunk * P.rows + row) * terms;
  for (int i = threadIdx.x; i < terms; i += blockDim.x) {
    const int o = i / kFit2Terms, t = i - o * kFit2Terms;
    const int li = o * kFit2Stride + t;
    double s = f2s[li];
    for (int w = 1; w < nwv; ++w) s += f2s[(int64_t)w * per + li];
    dst[i] = s;
  }
  // pair counts: integer sums, exact in any order
  for (int g = threadIdx.x; g < P.groups; g += blockDim.x)
    if (cnt[g]) atomicAdd(&P.pairs[g], cnt[g]);
}

// chunk sums in chunk order: sums[row][i] = sum over c of part[c][row][i]
__global__ void fit2_chunks_kernel(const double* part, double* sums, int chunks, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < chunks; ++c) s += part[(int64_t)c * n + i];
    sums[i] = s;
  }
}

// band entry (a, a + k) and right-side entry a of every group from the
// per-origin sums: the sum over the origins whose 4 x 4 patch holds both
// coefficients, in origin order (row, then m0); every entry written
__global__ void fit2_gather_kernel(const double* sums, double* band, double* rhs, int rows, int no,
                                   int groups, int nc0, int nc, int bw) {
  const int W = bw + 1;
  const int64_t per = (int64_t)nc * (W + 1);
  const int64_t total = (int64_t)groups * per;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(idx / per);
    const int64_t rem = idx - (int64_t)g * per;
    const int a = (int)(rem / (W + 1)), k = (int)(rem - (int64_t)a * (W + 1));
    const int ra = a / nc0, ca = a - ra * nc0;
    const double* sg = sums + (int64_t)g * no * kFit2Terms;
    const int64_t rstride = (int64_t)groups * no * kFit2Terms;
    double s = 0.0;
    if (k < W) {
      const int b = a + k;
      if (b < nc) {
        const int rb = b / nc0, cb = b - rb * nc0;
        const int rlo = (ra > rb ? ra : rb) - 3, rhi = ra < rb ? ra : rb;
        const int clo = (ca > cb ? ca : cb) - 3, chi = ca < cb ? ca : cb;
        for (int r = rlo < 0 ? 0 : rlo; r <= (rhi < rows - 1 ? rhi : rows - 1); ++r)
          for (int m0 = clo < 0 ? 0 : clo; m0 <= (chi < no - 1 ? chi : no - 1); ++m0) {
            const int i = 4 * (ra - r) + (ca - m0), j = 4 * (rb - r) + (cb - m0);
            const int t = 16 * i - i * (i - 1) / 2 + (j - i);
            s += sg[r * rstride + (int64_t)m0 * kFit2Terms + t];
          }
      }
      band[((int64_t)g * nc + a) * W + k] = s;
    } else {
      for (int r = ra - 3 < 0 ? 0 : ra - 3; r <= (ra < rows - 1 ? ra : rows - 1); ++r)
        for (int m0 = ca - 3 < 0 ? 0 : ca - 3; m0 <= (ca < no - 1 ? ca : no - 1); ++m0)
          s += sg[r * rstride + (int64_t)m0 * kFit2Terms + 136 + 4 * (ra - r) + (ca - m0)];
      rhs[(int64_t)g * nc + a] = s;
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

// The same factorisation and solves with the rows of U that column j
// reads (k in [j - bw, j]) in an LDS window of bw + 1 slots (row k at slot
// k mod (bw + 1)); the forward solve runs with the factorisation, and the
// backward solve reads U's rows back from global memory one row ahead.
// The arithmetic and its order are those of fit2_solve_kernel.
__global__ void __launch_bounds__(64) fit2_solve_lds_kernel(Solve2P P) {
#pragma clang fp contract(off)
  extern __shared__ double f2w[];
  const int lane = threadIdx.x, gr = blockIdx.x;
  const int nc = P.nc, bw = P.bw, W = bw + 1;
  double* win = f2w;                     // [W][W]
  double* yc = f2w + (int64_t)W * W;     // [nc]: y, then the solution
  double* U = P.band + (int64_t)gr * nc * W;
  const double* v = P.rhs + (int64_t)gr * nc;
  double tr = 0.0;
  for (int i = lane; i < nc; i += 64) tr += U[(int64_t)i * W];
  tr = wave_sum(tr);
  const double lam = P.ridge * (tr / nc);
  int sj = 0;   // j mod W
  for (int j = 0; j < nc; ++j) {
    double* wj = win + sj * W;
    for (int o = lane; o < W; o += 64) {
      const double a = U[(int64_t)j * W + o];
      wj[o] = o == 0 ? a + lam : a;
    }
    __syncthreads();
    const int k0 = j - bw > 0 ? j - bw : 0;
    const int s0 = sj - (j - k0) < 0 ? sj - (j - k0) + W : sj - (j - k0);   // k0 mod W
    double s = 0.0, sy = 0.0;
    {
      int sk = s0 + lane >= W ? s0 + lane - W : s0 + lane;
      for (int k = k0 + lane; k < j; k += 64) {
        const double u = win[sk * W + (j - k)];
        s += u * u;
        sy += u * yc[k];
        sk += 64;
        while (sk >= W) sk -= W;
      }
    }
    s = wave_sum(s);
    sy = wave_sum(sy);
    const double dj = wj[0] - s;
    const double d = dj > 0.0 ? sqrt(dj) : __builtin_nan("");
    const int i1 = j + bw < nc - 1 ? j + bw : nc - 1;
    for (int i = j + 1 + lane; i <= i1; i += 64) {
      const int kk = i - bw > 0 ? i - bw : 0;
      const int kb = kk > k0 ? kk : k0;
      double t = wj[i - j];
      int sk = s0 + (kb - k0);
      if (sk >= W) sk -= W;
      for (int k = kb; k < j; ++k) {
        t -= win[sk * W + (j - k)] * win[sk * W + (i - k)];
        if (++sk == W) sk = 0;
      }
      const double uji = t / d;
      wj[i - j] = uji;
      U[(int64_t)j * W + (i - j)] = uji;
    }
    if (lane == 0) {
      U[(int64_t)j * W] = d;
      yc[j] = (v[j] - sy) / d;
    }
    __syncthreads();
    wj[0] = d;
    if (++sj == W) sj = 0;
    __syncthreads();
  }
  // U c = y, rows of U read one step ahead
  constexpr int R = 3;   // W <= 3 * 64 + 1
  double ur[R], dg = 0.0;
  auto load_row = [&](int j, double (&u)[R], double& dd) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int o = 1 + lane + 64 * r;
      u[r] = (j >= 0 && o < W) ? U[(int64_t)j * W + o] : 0.0;
    }
    dd = j >= 0 ? U[(int64_t)j * W] : 1.0;
  };
  load_row(nc - 1, ur, dg);
  for (int j = nc - 1; j >= 0; --j) {
    double un[R], dn;
    load_row(j - 1, un, dn);
    const int i1 = j + bw < nc - 1 ? j + bw : nc - 1;
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = j + 1 + lane + 64 * r;
      if (i <= i1) s += ur[r] * yc[i];
    }
    s = wave_sum(s);
    if (lane == 0) yc[j] = (yc[j] - s) / dg;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) ur[r] = un[r];
    dg = dn;
  }
  double* c = P.coef + (int64_t)gr * nc;
  for (int i = lane; i < nc; i += 64) c[i] = yc[i];
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
  if (isnan(cfg->ev_z_lo) || isnan(cfg->ev_z_hi))
    return set_error(ANTS_E_ARG, "%s: depth window bound is NaN", who);
  if (cfg->d_base) {
    if (cfg->kind != ANTS_LRF_XY)
      return set_error(ANTS_E_ARG, "%s: an axial base is for XY residual fits", who);
    if (cfg->base_nb < 2 || cfg->base_nb > 256)
      return set_error(ANTS_E_ARG, "%s: base_nb = %d outside 2..256", who, cfg->base_nb);
    if (!(cfg->base_lo >= 0.0 && cfg->base_hi > cfg->base_lo && isfinite(cfg->base_hi)))
      return set_error(ANTS_E_ARG, "%s: base domain [%g, %g] invalid", who, cfg->base_lo,
                       cfg->base_hi);
  }
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
  const int rows = cfg->nb[1] - 1, no = cfg->nb[0] - 1;
  // row accumulation when two waves' copies of a row's sums fit in LDS
  const size_t per_wave = (size_t)n_groups * no * kFit2Stride * sizeof(double);
  const size_t cnt_bytes = (size_t)n_groups * sizeof(unsigned long long);
  int nwv = 0;
  for (int w = 4; w >= 2 && !nwv; w >>= 1)
    if (w * per_wave + cnt_bytes <= (size_t)kFit2LdsBytes) nwv = w;
  int chunks = 0;
  int64_t chunk_len = 0;
  if (nwv && n_events > 0) {
    const int64_t tile = 64 * nwv;
    const int64_t want = ((int64_t)num_cu() * 4 + rows - 1) / rows;
    chunk_len = (n_events + want - 1) / want;
    chunk_len = (chunk_len + tile - 1) / tile * tile;
    chunks = (int)((n_events + chunk_len - 1) / chunk_len);
  }
  const int64_t terms = (int64_t)n_groups * no * kFit2Terms;
  const size_t nband = (size_t)n_groups * nc * (bw + 1), nrhs = (size_t)n_groups * nc;
  const size_t zbytes = (nband + 2 * nrhs) * sizeof(double) +
                        ((size_t)n_groups + 1) * sizeof(unsigned long long);
  const size_t zpad = (zbytes + 255) / 256 * 256;
  const size_t pbytes = chunks ? (size_t)(chunks + 1) * rows * terms * sizeof(double) : 0;
  hipError_t e = ensure(&set->ws_fit2, &set->ws_fit2_bytes, zpad + pbytes);
  if (e != hipSuccess) return hip_error(e, who);
  double* band = (double*)set->ws_fit2;
  double* rhs = band + nband;
  double* ywork = rhs + nrhs;
  unsigned long long* pairs = (unsigned long long*)(ywork + nrhs);
  unsigned long long* used = pairs + n_groups;
  double* part = (double*)((char*)set->ws_fit2 + zpad);
  double* sums = part + (size_t)chunks * rows * terms;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t nz = (int64_t)(zbytes / sizeof(double));
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
    P.base = cfg->d_base;
    P.base_nb = cfg->base_nb;
    P.base_lo = cfg->base_lo;
    P.base_hi = cfg->base_hi;
    P.base_inv = cfg->d_base ? (double)(cfg->base_nb - 1) / (cfg->base_hi - cfg->base_lo) : 0.0;
    P.zwin = cfg->ev_z_lo < cfg->ev_z_hi;
    P.zw_lo = cfg->ev_z_lo;
    P.zw_hi = cfg->ev_z_hi;
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
    P.rows = rows;
    P.no = no;
    P.chunks = chunks;
    P.chunk_len = chunk_len;
    P.part = part;
    if (nwv) {
      const size_t smem = nwv * per_wave + cnt_bytes;
      e = hipFuncSetAttribute((const void*)fit2_rows_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
      if (e != hipSuccess) return hip_error(e, who);
      hipLaunchKernelGGL(fit2_rows_kernel, dim3((unsigned)(rows * chunks)), dim3(64 * nwv), smem,
                         s, P);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_error(e, who);
      const int64_t nsum = (int64_t)rows * terms;
      hipLaunchKernelGGL(fit2_chunks_kernel,
                         dim3((unsigned)std::min<int64_t>((nsum + 255) / 256, 4096)), dim3(256), 0,
                         s, (const double*)part, sums, chunks, nsum);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_error(e, who);
      const int64_t ng = (int64_t)n_groups * nc * (bw + 2);
      hipLaunchKernelGGL(fit2_gather_kernel,
                         dim3((unsigned)std::min<int64_t>((ng + 255) / 256, 4096)), dim3(256), 0,
                         s, (const double*)sums, band, rhs, rows, no, n_groups, nc0, nc, bw);
    } else {
      int64_t blocks = (n_events + 3) / 4;
      const int64_t cap = (int64_t)num_cu() * 8;
      if (blocks > cap) blocks = cap;
      hipLaunchKernelGGL(fit2_accum_kernel, dim3((unsigned)blocks), dim3(256), 0, s, P);
    }
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
  const size_t wbytes = ((size_t)(bw + 1) * (bw + 1) + nc) * sizeof(double);
  if (bw + 1 <= 3 * 64 + 1 && wbytes <= (size_t)kFit2LdsBytes) {
    e = hipFuncSetAttribute((const void*)fit2_solve_lds_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)wbytes);
    if (e != hipSuccess) return hip_error(e, who);
    hipLaunchKernelGGL(fit2_solve_lds_kernel, dim3(n_groups), dim3(64), wbytes, s, S);
  } else {
    hipLaunchKernelGGL(fit2_solve_kernel, dim3(n_groups), dim3(64), 0, s, S);
  }
  e = hipGetLastError();
  return e == hipSuccess ? ANTS_OK : hip_error(e, who);
}
