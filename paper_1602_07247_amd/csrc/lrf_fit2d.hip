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
// of an event has the same m1 (its row).  The kept events are bucketed by
// row (a stable counting sort: counts per event chunk, offsets, scatter in
// event order).  Blocks own one row, one segment of its events and one
// batch of groups (as many as two waves' LDS copies of the row's
// per-origin sums hold: 152 FP64 per origin and group); lanes take (event,
// member sensor) pairs and each wave adds them into its own copy.  The
// block adds its waves' copies in wave order, a second kernel the segments
// in segment order, and each band entry is the sum over the origins that
// hold it, in origin order: the same bits on every call.
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
  int nb0, nb1;
  double lo0, hi0, lo1, hi1, inv_d0, inv_d1;
  const int32_t* group;   // per sensor index
  int groups;
  unsigned long long* pairs;   // [groups]
  unsigned long long* used;    // [1]
  // row accumulation: rows = nb1 - 1, no = nb0 - 1 origins per row
  int rows, no;
  double* part;        // [segments][rows][groups * no * kFit2Terms]
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

// ---- events bucketed by row (a stable counting sort), then blocks (row,
// segment of the row's events, batch of groups) with lanes over (event,
// member sensor) pairs

// the event's row (the interval of its z or y), or -1 when it is not kept
// or lies outside the second axis' domain
__device__ __forceinline__ int fit2_event_row(const Fit2P& P, int64_t e, bool& kept) {
  kept = fit2_keep(P, e);
  if (!kept) return -1;
  double w = P.rz ? (double)P.z[e] : (double)P.y[e];
  if (!P.rz && P.shift) w += (double)P.shift[2 * e + 1];
  int m1;
  double t1;
  return locate64(w, P.nb1, P.lo1, P.hi1, P.inv_d1, m1, t1) ? m1 : -1;
}

// per event chunk: kept events (added to used) and events per row
__global__ void __launch_bounds__(256) fit2_rowcount_kernel(Fit2P P, int* cnt, int64_t clen) {
  __shared__ int h[kFit2MaxKnots];
  __shared__ unsigned long long kept_sum;
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < P.rows; i += blockDim.x) h[i] = 0;
  if (threadIdx.x == 0) kept_sum = 0ull;
  __syncthreads();
  const int64_t e0 = (int64_t)c * clen, e1 = e0 + clen < P.n ? e0 + clen : P.n;
  unsigned long long kept_n = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    bool kept;
    const int r = fit2_event_row(P, e, kept);
    kept_n += kept ? 1ull : 0ull;
    if (r >= 0) atomicAdd(&h[r], 1);
  }
  atomicAdd(&kept_sum, kept_n);
  __syncthreads();
  for (int i = threadIdx.x; i < P.rows; i += blockDim.x) cnt[(int64_t)c * P.rows + i] = h[i];
  if (threadIdx.x == 0 && kept_sum) atomicAdd(P.used, kept_sum);
}

// offsets: row r's events start at rstart[r]; chunk c's events of row r at
// off[c][r] (rows in order, chunks in order within a row)
__global__ void __launch_bounds__(64) fit2_rowscan_kernel(const int* cnt, int* off, int* rstart,
                                                          int rows, int cchunks) {
  __shared__ int tot[kFit2MaxKnots];
  const int r = threadIdx.x;
  if (r < rows) {
    int t = 0;
    for (int c = 0; c < cchunks; ++c) t += cnt[(int64_t)c * rows + r];
    tot[r] = t;
  }
  __syncthreads();
  if (r < rows) {
    int base = 0;
    for (int q = 0; q < r; ++q) base += tot[q];
    rstart[r] = base;
    if (r == rows - 1) rstart[rows] = base + tot[r];
    for (int c = 0; c < cchunks; ++c) {
      off[(int64_t)c * rows + r] = base;
      base += cnt[(int64_t)c * rows + r];
    }
  }
}

// one wave per event chunk: events to their row's list in event order
__global__ void __launch_bounds__(64) fit2_rowscatter_kernel(Fit2P P, const int* off,
                                                             int* sorted, int64_t clen) {
  __shared__ int run[kFit2MaxKnots];
  const int lane = threadIdx.x, c = blockIdx.x;
  for (int i = lane; i < P.rows; i += 64) run[i] = off[(int64_t)c * P.rows + i];
  __syncthreads();
  const int64_t e0 = (int64_t)c * clen, e1 = e0 + clen < P.n ? e0 + clen : P.n;
  const uint64_t lt = (1ull << lane) - 1ull;
  for (int64_t base = e0; base < e1; base += 64) {
    const int64_t e = base + lane;
    int r = -1;
    if (e < e1) {
      bool kept;
      r = fit2_event_row(P, e, kept);
    }
    uint64_t left = __ballot(r >= 0);
    while (left) {
      const int l = __builtin_ctzll(left);
      const int r0 = __shfl(r, l);
      const uint64_t m = __ballot(r == r0);
      const int b0 = run[r0];
      if (r == r0) sorted[b0 + __popcll(m & lt)] = (int)e;
      __syncthreads();
      if (lane == 0) run[r0] = b0 + __popcll(m);
      __syncthreads();
      left &= ~m;
    }
  }
}

// block (row, segment, batch): the batch's members are the active sensors
// whose group lies in [g0, g0 + gb), in sensor order; the block's waves
// take consecutive parts of the segment, pairs in member-major order, each
// wave summing into its own LDS copy
// acc[((group - g0) * no + m0) * kFit2Stride + term], then the block adds
// them in wave order to part[seg][row][group][m0][term]
__global__ void __launch_bounds__(128) fit2_rowsort_kernel(Fit2P P, const int* sorted,
                                                           const int* rstart, int segs, int gb) {
  extern __shared__ double f2s[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int row = blockIdx.x % P.rows;
  const int seg = (blockIdx.x / P.rows) % segs;
  const int batch = blockIdx.x / (P.rows * segs);
  const int g0 = batch * gb;
  const int gn = P.groups - g0 < gb ? P.groups - g0 : gb;
  const int per = gb * P.no * kFit2Stride;
  double* acc = f2s + (int64_t)wave * per;
  unsigned long long* cnt = (unsigned long long*)(f2s + (int64_t)nwv * per);
  int* mem = (int*)(cnt + gb);   // [kMaxSensors] member slots
  __shared__ int nm_s;
  for (int i = lane; i < per; i += 64) acc[i] = 0.0;
  for (int i = threadIdx.x; i < gb; i += blockDim.x) cnt[i] = 0ull;
  if (threadIdx.x == 0) {
    int k = 0;
    for (int a = 0; a < P.na; ++a) {
      const int gr = P.group[P.col[a]];
      if (gr >= g0 && gr < g0 + gn) mem[k++] = a;
    }
    nm_s = k;
  }
  __syncthreads();
  const int nm = nm_s;
  const int rs = rstart[row], rl = rstart[row + 1] - rs;
  const int sl = (rl + segs - 1) / segs;
  const int s0 = rs + seg * sl;
  const int s1 = s0 + sl < rs + rl ? s0 + sl : rs + rl;
  if (nm > 0 && s1 > s0) {
    const int wl = (s1 - s0 + nwv - 1) / nwv;
    const int w0 = s0 + wave * wl;
    const int w1 = w0 + wl < s1 ? w0 + wl : s1;
    const int ne = w1 > w0 ? w1 - w0 : 0;
    const int64_t np = (int64_t)ne * nm;
    // XY: pairs member-major, so the lanes of a pass hold different events
    // (one event's pairs share its origin); r-z: event-major, the sensors
    // of one event lie at different distances
    for (int64_t p = lane; p < np; p += 64) {
      int i, j;
      if (P.rz) {
        i = (int)(p / nm);
        j = (int)(p - (int64_t)i * nm);
      } else {
        j = (int)(p / ne);
        i = (int)(p - (int64_t)j * ne);
      }
      const int64_t ev = sorted[w0 + i];
      const int a = mem[j];
      const int col = P.col[a];
      double xe = P.x[ev], ye = P.y[ev];
      if (P.shift) {
        xe += (double)P.shift[2 * ev];
        ye += (double)P.shift[2 * ev + 1];
      }
      const double w = P.rz ? (double)P.z[ev] : ye;
      double u;
      if (P.rz) {
        const double dx = xe - P.X[a], dy = ye - P.Y[a];
        u = sqrt(dx * dx + dy * dy);
      } else {
        u = xe;
      }
      int m0, m1;
      double t0, t1;
      if (!locate64(u, P.nb0, P.lo0, P.hi0, P.inv_d0, m0, t0)) continue;
      if (!locate64(w, P.nb1, P.lo1, P.hi1, P.inv_d1, m1, t1)) continue;   // in the row
      double b0[4], b1[4];
      bweights64(t0, b0);
      bweights64(t1, b1);
      double tg = (double)P.sig[ev * P.ld + col] / ((double)P.E[ev] * P.g[a]);
      if (P.base) {
        const double dx = xe - P.X[a], dy = ye - P.Y[a];
        tg -= base_value(P, sqrt(dx * dx + dy * dy));
      }
      double wt[16];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int pp = 0; pp < 4; ++pp) wt[4 * q + pp] = b1[q] * b0[pp];
      const int gl = P.group[col] - g0;
      double* o = acc + (gl * P.no + m0) * kFit2Stride;
      int k = 0;
#pragma unroll
      for (int ii = 0; ii < 16; ++ii)
#pragma unroll
        for (int jj = ii; jj < 16; ++jj) atomicAdd(&o[k++], wt[ii] * wt[jj]);
#pragma unroll
      for (int ii = 0; ii < 16; ++ii) atomicAdd(&o[136 + ii], wt[ii] * tg);
      atomicAdd(&cnt[gl], 1ull);
    }
  }
  __syncthreads();
  const int64_t terms = (int64_t)P.groups * P.no * kFit2Terms;
  double* dst = P.part + ((int64_t)seg * P.rows + row) * terms + (int64_t)g0 * P.no * kFit2Terms;
  const int bterms = gn * P.no * kFit2Terms;
  for (int i = threadIdx.x; i < bterms; i += blockDim.x) {
    const int o = i / kFit2Terms, t = i - o * kFit2Terms;
    const int li = o * kFit2Stride + t;
    double s = f2s[li];
    for (int w = 1; w < nwv; ++w) s += f2s[(int64_t)w * per + li];
    dst[i] = s;
  }
  for (int g = threadIdx.x; g < gn; g += blockDim.x)
    if (cnt[g]) atomicAdd(&P.pairs[g0 + g], cnt[g]);
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
  // row j of A is read one column ahead (registers), so its memory latency
  // overlaps the previous column's work
  constexpr int RA = 4;   // W <= 4 * 64
  double ra[RA];
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    const int o = lane + 64 * r;
    ra[r] = o < W ? U[o] : 0.0;
  }
  int sj = 0;   // j mod W
  for (int j = 0; j < nc; ++j) {
    double* wj = win + sj * W;
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int o = lane + 64 * r;
      if (o < W) wj[o] = o == 0 ? ra[r] + lam : ra[r];
    }
    if (j + 1 < nc) {
#pragma unroll
      for (int r = 0; r < RA; ++r) {
        const int o = lane + 64 * r;
        ra[r] = o < W ? U[(int64_t)(j + 1) * W + o] : 0.0;
      }
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
      // k = kb .. j - 1 in order; along k both operands step by W - 1 in
      // the window until the slot wraps to 0 (two linear runs)
      const int n = j - kb;
      const int n1 = n < W - sk ? n : W - sk;
      const double* pa = win + sk * W + (j - kb);
      const double* pb = win + sk * W + (i - kb);
#pragma unroll 8
      for (int q = 0; q < n1; ++q) t -= pa[q * (W - 1)] * pb[q * (W - 1)];
      pa = win + (j - kb - n1);
      pb = win + (i - kb - n1);
#pragma unroll 8
      for (int q = 0; q < n - n1; ++q) t -= pa[q * (W - 1)] * pb[q * (W - 1)];
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
  // events bucketed by row; batches of gb groups on two waves, segs
  // segments per row; cchunks event chunks of clen for the bucketing
  const size_t sort_fixed = kMaxSensors * sizeof(int) + 64;
  const size_t per_group = (size_t)no * kFit2Stride * sizeof(double);
  int gb = 0, nbatch = 0, segs = 0, cchunks = 0;
  int64_t clen = 0;
  if (n_events > 0) {
    if (n_events > INT32_MAX)
      return set_error(ANTS_E_UNSUPPORTED, "%s: more than 2^31 - 1 events", who);
    gb = (int)(((size_t)kFit2LdsBytes - sort_fixed) / (2 * per_group + sizeof(unsigned long long)));
    if (gb > n_groups) gb = n_groups;
    if (gb < 1) return set_error(ANTS_E_UNSUPPORTED, "%s: nb[0] = %d too large", who, cfg->nb[0]);
    nbatch = (n_groups + gb - 1) / gb;
    segs = (int)(((int64_t)num_cu() * 4 + (int64_t)rows * nbatch - 1) / ((int64_t)rows * nbatch));
    segs = segs < 1 ? 1 : (segs > 64 ? 64 : segs);
    clen = (n_events + 1023) / 1024;
    clen = clen < 1024 ? 1024 : clen;
    clen = (clen + 255) / 256 * 256;
    cchunks = (int)((n_events + clen - 1) / clen);
  }
  const int64_t terms = (int64_t)n_groups * no * kFit2Terms;
  const size_t nband = (size_t)n_groups * nc * (bw + 1), nrhs = (size_t)n_groups * nc;
  const size_t zbytes = (nband + 2 * nrhs) * sizeof(double) +
                        ((size_t)n_groups + 1) * sizeof(unsigned long long);
  const size_t zpad = (zbytes + 255) / 256 * 256;
  const size_t pbytes = segs ? (size_t)(segs + 1) * rows * terms * sizeof(double) : 0;
  const size_t ibytes = cchunks ? ((size_t)2 * cchunks * rows + rows + 1 + (size_t)n_events) *
                                      sizeof(int) : 0;
  hipError_t e = ensure(&set->ws_fit2, &set->ws_fit2_bytes, zpad + pbytes + ibytes);
  if (e != hipSuccess) return hip_error(e, who);
  double* band = (double*)set->ws_fit2;
  double* rhs = band + nband;
  double* ywork = rhs + nrhs;
  unsigned long long* pairs = (unsigned long long*)(ywork + nrhs);
  unsigned long long* used = pairs + n_groups;
  double* part = (double*)((char*)set->ws_fit2 + zpad);
  double* sums = part + (size_t)segs * rows * terms;
  int* rcnt = (int*)((char*)set->ws_fit2 + zpad + pbytes);
  int* roff = rcnt + (size_t)cchunks * rows;
  int* rstart = roff + (size_t)cchunks * rows;
  int* sorted = rstart + rows + 1;
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
    P.lo0 = cfg->lo[0];
    P.hi0 = cfg->hi[0];
    P.lo1 = cfg->lo[1];
    P.hi1 = cfg->hi[1];
    P.inv_d0 = (double)(cfg->nb[0] - 1) / (cfg->hi[0] - cfg->lo[0]);
    P.inv_d1 = (double)(cfg->nb[1] - 1) / (cfg->hi[1] - cfg->lo[1]);
    P.group = d_group;
    P.groups = n_groups;
    P.pairs = pairs;
    P.used = used;
    P.rows = rows;
    P.no = no;
    P.part = part;
    {
      hipLaunchKernelGGL(fit2_rowcount_kernel, dim3((unsigned)cchunks), dim3(256), 0, s, P, rcnt,
                         clen);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_error(e, who);
      hipLaunchKernelGGL(fit2_rowscan_kernel, dim3(1), dim3(64), 0, s, (const int*)rcnt, roff,
                         rstart, rows, cchunks);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_error(e, who);
      hipLaunchKernelGGL(fit2_rowscatter_kernel, dim3((unsigned)cchunks), dim3(64), 0, s, P,
                         (const int*)roff, sorted, clen);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_error(e, who);
      const size_t smem = 2 * gb * per_group + gb * sizeof(unsigned long long) + sort_fixed;
      e = hipFuncSetAttribute((const void*)fit2_rowsort_kernel,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
      if (e != hipSuccess) return hip_error(e, who);
      hipLaunchKernelGGL(fit2_rowsort_kernel, dim3((unsigned)(rows * segs * nbatch)), dim3(128),
                         smem, s, P, (const int*)sorted, (const int*)rstart, segs, gb);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_error(e, who);
      const int64_t nsum = (int64_t)rows * terms;
      hipLaunchKernelGGL(fit2_chunks_kernel,
                         dim3((unsigned)std::min<int64_t>((nsum + 255) / 256, 4096)), dim3(256), 0,
                         s, (const double*)part, sums, segs, nsum);
      e = hipGetLastError();
      if (e != hipSuccess) return hip_error(e, who);
      const int64_t ng = (int64_t)n_groups * nc * (bw + 2);
      hipLaunchKernelGGL(fit2_gather_kernel,
                         dim3((unsigned)std::min<int64_t>((ng + 255) / 256, 4096)), dim3(256), 0,
                         s, (const double*)sums, band, rhs, rows, no, n_groups, nc0, nc, bw);
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
