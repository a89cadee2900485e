// Contracting-grid reconstruction kernel for gfx950 (CDNA4, wave64).
//
// Method (arXiv:1602.07247, Sec. 5.1.2.2): per event, a regular grid of
// nodes centred on the start position; at every node the expected signals
// come from the sensors' light response functions, the energy is the ratio
// of the summed signals to the summed LRFs, the match is scored by maximum
// likelihood or least squares (Sec. 5.1.2), the best node becomes the centre
// of a finer grid with the same node count, for a fixed number of
// iterations.  Start: gain-weighted centroid (Sec. 5.1.1) or the strongest
// sensor (Sec. 5.1.2.1) or a caller seed.  Passive sensors are skipped
// (Sec. 5.3).
//
// Mapping: one wavefront per event, lanes = grid nodes (tiles of 64 nodes),
// a uniform loop over the event's active sensors.  Per-event sensor records
// are broadcast from LDS; LRF piecewise-cubic tables sit in LDS (axial and
// r-z; the r-z table is collapsed along z for the z-planes of each
// iteration so each (node, sensor) pair costs one cubic in r); XY bicubic
// coefficients are read through the cache.  Variants of the screen:
//  - r-z, ML, 3/5/7 planes: lanes take (x-y column, sensor group) and one
//    distance serves every plane of the column (column-factored screen);
//  - grids of at most 32 nodes, or a last tile of at most 32 nodes: the
//    two half-waves take alternate sensors and add their sums.
//
// Precision: nodes are first screened in FP32 with the statistic written
// relative to the current centre (ratios L/L_centre and S/S_centre), which
// keeps the rounding error proportional to the distance from the centre.
// A per-iteration bound on that error is computed at the best screened
// node; every node whose screened value lies within (a multiple of) the
// bound of the best is re-evaluated in FP64 (the vector FP64 rate equals
// the unpacked FP32 rate on this chip), in lane groups sized by a cost
// model, and the FP64 values decide.  FP64 values within 1e-12 N of the
// best are ties, which go to the lowest node index.
#pragma once

#include <math.h>

#include "ants_internal.h"
#include "lrf64.h"

namespace ants {
namespace {

constexpr float kU = 5.9604645e-8f;  // unit roundoff of FP32
constexpr float kInf = __builtin_huge_valf();
constexpr float kLog2e = 1.4426950408889634f;
// Tie tolerance of the FP64 decisions, relative to the event's summed
// signal N: node statistics closer than this are equal, and the lowest node
// index wins (far above double rounding, far below real gaps between nodes).
constexpr double kTieRel = 1e-12;

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Cross-lane moves within rows of 16 lanes (DPP): xor 1, xor 2 (quad
// permutes), then the half-row and row mirrors, which act as xor 4 and xor 8
// once the quads, then the half-rows, hold equal values.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
template <int C>
__device__ __forceinline__ int dpp(int v) {
  return __builtin_amdgcn_mov_dpp(v, C, 0xF, 0xF, true);
}
template <int C>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(dpp<C>(__float_as_int(v)));
}
template <int C>
__device__ __forceinline__ double dpp(double v) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = dpp<C>(p.x);
  p.y = dpp<C>(p.y);
  return __builtin_bit_cast(double, p);
}
__device__ __forceinline__ float lane_val(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int lane_val(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double lane_val(double v, int l) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readlane(p.x, l);
  p.y = __builtin_amdgcn_readlane(p.y, l);
  return __builtin_bit_cast(double, p);
}
// Sums over the wave (all lanes active): butterfly within each row of 16
// lanes, then the four row sums in a fixed order; every lane gets the same
// value.
template <typename T>
__device__ __forceinline__ T wsum(T v) {
  v += dpp<kDppXor1>(v);
  v += dpp<kDppXor2>(v);
  v += dpp<kDppHalfMirror>(v);
  v += dpp<kDppMirror>(v);
  return ((lane_val(v, 0) + lane_val(v, 16)) + lane_val(v, 32)) + lane_val(v, 48);
}
// Sums over aligned groups of 2^lg lanes (lg uniform, all lanes active);
// every lane gets its group's sum.
template <typename T>
__device__ __forceinline__ T gsum(T v, int lg, int lane) {
  if (lg >= 1) v += dpp<kDppXor1>(v);
  if (lg >= 2) v += dpp<kDppXor2>(v);
  if (lg >= 3) v += dpp<kDppHalfMirror>(v);
  if (lg >= 4) v += dpp<kDppMirror>(v);
  if (lg == 5) {
    const T lo = lane_val(v, 0) + lane_val(v, 16), hi = lane_val(v, 32) + lane_val(v, 48);
    v = lane < 32 ? lo : hi;
  } else if (lg >= 6) {
    v = ((lane_val(v, 0) + lane_val(v, 16)) + lane_val(v, 32)) + lane_val(v, 48);
  }
  return v;
}
__device__ __forceinline__ double wsum_d(double v) { return wsum(v); }
__device__ __forceinline__ float wsum_f(float v) { return wsum(v); }
// lexicographic minimum of (value, index) over the wave; with MAX, maximum
// of the value with the lowest index among equal values
template <bool MAX, typename T>
__device__ __forceinline__ void take_better(T& v, int& j, T v2, int j2) {
  const bool b = MAX ? (v2 > v || (v2 == v && j2 < j)) : (v2 < v || (v2 == v && j2 < j));
  if (b) { v = v2; j = j2; }
}
template <bool MAX, typename T>
__device__ __forceinline__ void warg(T& v, int& j) {
  take_better<MAX>(v, j, dpp<kDppXor1>(v), dpp<kDppXor1>(j));
  take_better<MAX>(v, j, dpp<kDppXor2>(v), dpp<kDppXor2>(j));
  take_better<MAX>(v, j, dpp<kDppHalfMirror>(v), dpp<kDppHalfMirror>(j));
  take_better<MAX>(v, j, dpp<kDppMirror>(v), dpp<kDppMirror>(j));
  T v0 = lane_val(v, 0);
  int j0 = lane_val(j, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) take_better<MAX>(v0, j0, lane_val(v, r), lane_val(j, r));
  v = v0;
  j = j0;
}
__device__ __forceinline__ void wargmin_f(float& v, int& j) { warg<false>(v, j); }
__device__ __forceinline__ void wargmin_d(double& v, int& j) { warg<false>(v, j); }
// strongest sensor, lowest index among equals
__device__ __forceinline__ void wargmax_f(float& v, int& j) { warg<true>(v, j); }
__device__ __forceinline__ int prefix_count(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
// values equal in every lane, moved to scalar registers
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uni(double v) {
  int2 p = __builtin_bit_cast(int2, v);
  p.x = __builtin_amdgcn_readfirstlane(p.x);
  p.y = __builtin_amdgcn_readfirstlane(p.y);
  return __builtin_bit_cast(double, p);
}
// An opaque copy of a value: stops the compiler from hoisting per-lane
// set-up work out of the event loop and pinning it in registers for the
// whole kernel (it is cheaper to recompute than to keep).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// FP64 r-z LRF of sensor a at (x, y) on a z-plane whose B-spline rows were
// collapsed along z beforehand (zc: nc0 coefficients of the 1-D spline in r)
__device__ __forceinline__ double lrf64_plane(const DevLrf& L, double X, double Y, double x,
                                              double y, const double* zc) {
  const double dx = x - X, dy = y - Y;
  const double r = sqrt(dx * dx + dy * dy);
  const double tol = 1e-9 * (L.hi0 - L.lo0);
  if (!(r >= L.lo0 - tol && r <= L.hi0 + tol)) return 0.0;
  const double v = (r - L.lo0) * L.inv_d0;
  int k = (int)floor(v);
  k = k < 0 ? 0 : k;
  k = k > L.nb0 - 2 ? L.nb0 - 2 : k;
  double b[4];
  bweights64(v - (double)k, b);
  const double val = zc[k] * b[0] + zc[k + 1] * b[1] + zc[k + 2] * b[2] + zc[k + 3] * b[3];
  return val > 0.0 ? val : 0.0;
}

// --------------------------------------------------- FP32 screening LRF

// Per-lane description of one node for the FP32 screen.
template <int KIND>
struct NodeF {
  float ox, oy;          // offset from the centre (axial, r-z)
  const float4* tab;     // r-z: this node's z-plane table (LDS)
};
template <>
struct NodeF<ANTS_LRF_XY> {
  int cell;              // my * nc0 + mx
  float w[16];           // wy[a] * wx[b]
};
template <>
struct NodeF<ANTS_LRF_COMPOSITE> {
  float ox, oy;          // offset from the centre (axial part)
  int cell;              // residual: my * xnc0 + mx
  float w[16];           // residual weights (0 outside the residual's domain)
};
template <>
struct NodeF<ANTS_LRF_SLICED> {
  int cell;              // lower plane p * pstride + my * nc0 + mx
  int pstride;           // coefficients per plane
  float t;               // position between plane p and p + 1
  float w[16];
};

// Radial kinds: node-sensor distance in units of the breakpoint spacing
// (v = r / d0, the domain starting at r = 0), the sensor's table (r-z: the
// node's plane table) and the cubic piece at v; index nlast is an all-zero
// interval past the end of the domain.
template <int KIND>
__device__ __forceinline__ float rad_v(const NodeF<KIND>& nd, float dX, float dY) {
  const float dx = nd.ox - dX, dy = nd.oy - dY;
  return __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
}
template <int KIND>
__device__ __forceinline__ const float4* rad_tab(const NodeF<KIND>& nd, const float4* btab,
                                                 int tofs) {
  if constexpr (KIND == ANTS_LRF_RZ) return nd.tab;
  else return btab + tofs;
}
template <bool NN>
__device__ __forceinline__ float rad32(const float4* T, float v, int nlast) {
  const int m = (int)fminf(v, (float)nlast);
  const float t = __builtin_amdgcn_fractf(v);
  const float4 c = T[m];
  const float p = fmaf(fmaf(fmaf(c.w, t, c.z), t, c.y), t, c.x);
  return NN ? p : fmaxf(p, 0.f);
}

// FP32 bicubic of a 4 x 4 coefficient patch (rows nc0 apart) with the
// node's weights, read through the cache
__device__ __forceinline__ float bicubic32(const float* p, int nc0, const float (&w)[16]) {
  typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
  f4u r0 = *(const f4u*)(p);
  f4u r1 = *(const f4u*)(p + nc0);
  f4u r2 = *(const f4u*)(p + 2 * nc0);
  f4u r3 = *(const f4u*)(p + 3 * nc0);
  float v = w[0] * r0.x;
  v = fmaf(w[1], r0.y, v);
  v = fmaf(w[2], r0.z, v);
  v = fmaf(w[3], r0.w, v);
  v = fmaf(w[4], r1.x, v);
  v = fmaf(w[5], r1.y, v);
  v = fmaf(w[6], r1.z, v);
  v = fmaf(w[7], r1.w, v);
  v = fmaf(w[8], r2.x, v);
  v = fmaf(w[9], r2.y, v);
  v = fmaf(w[10], r2.z, v);
  v = fmaf(w[11], r2.w, v);
  v = fmaf(w[12], r3.x, v);
  v = fmaf(w[13], r3.y, v);
  v = fmaf(w[14], r3.z, v);
  v = fmaf(w[15], r3.w, v);
  return v;
}

// FP32 coefficient tables and row length the screen's bicubics read
// (composite: its XY residual)
template <int KIND>
__device__ __forceinline__ const float* scr_c32(const DevLrf& L) {
  return KIND == ANTS_LRF_COMPOSITE ? L.xc32 : L.c32;
}
template <int KIND>
__device__ __forceinline__ int scr_nc0(const DevLrf& L) {
  return KIND == ANTS_LRF_COMPOSITE ? L.xnc0 : L.nc0;
}

// Sensor record broadcast from LDS: A = {dX, dY, n, 1/L_c}, B = {g, L_c, table offset, a}
template <int KIND, bool NN>
__device__ __forceinline__ float lrf32(const NodeF<KIND>& nd, float dX, float dY, int tofs,
                                       const float4* btab, const float* c32, int nc0,
                                       float finv, int nlast) {
  if constexpr (KIND == ANTS_LRF_XY) {
    return fmaxf(bicubic32(c32 + tofs + nd.cell, nc0, nd.w), 0.f);
  } else if constexpr (KIND == ANTS_LRF_COMPOSITE) {
    // the shared axial table (row 0) plus the sensor's residual, clamped
    const float a = rad32<true>(btab, rad_v(nd, dX, dY), nlast);
    return fmaxf(a + bicubic32(c32 + tofs + nd.cell, nc0, nd.w), 0.f);
  } else if constexpr (KIND == ANTS_LRF_SLICED) {
    const float* p = c32 + tofs + nd.cell;
    const float a = fmaxf(bicubic32(p, nc0, nd.w), 0.f);
    const float b = fmaxf(bicubic32(p + nd.pstride, nc0, nd.w), 0.f);
    return fmaf(nd.t, b - a, a);
  } else {
    const float v = rad_v(nd, dX, dY);
    return rad32<NN>(rad_tab<KIND>(nd, btab, tofs), v, nlast);
  }
}

// Node j of the current grid: FP64 position, FP32 screen description and
// validity (nodes whose z, or XY position, leave the LRF domain have S = 0).
// Node index -> (jx, jy, jz) packed as jx | jy << shy | jz << shz (16 bits),
// one entry per node lane (avoids integer division in the loops).
__device__ __forceinline__ void fill_nodeidx(const GridP& G, uint16_t* tab, int ntab, int lane) {
  for (int j = lane; j < ntab; j += 64) {
    int v = 0;
    if (j < G.nn) {
      const int jx = j % G.nx, jy = (j / G.nx) % G.ny, jz = j / (G.nx * G.ny);
      v = jx | (jy << G.shy) | (jz << G.shz);
    }
    tab[j] = (uint16_t)v;
  }
}

// FP64 data of an active sensor, stored per event in sensor order (the
// FP32 records are re-ordered every iteration).
struct SensorRec64 {
  double X, Y, g;
  int coff;            // FP64 coefficient offset
  float n;             // signal
};

// A wave's LDS area (sizes as in wave_lds_bytes).
struct WaveLds {
  float4* recA;        // per sensor record: dX, dY, n, 1/L_c
  float4* recB;        // g, L_c, table offset, sensor index
  SensorRec64* rec64;  // X, Y, g, FP64 coefficient offset, signal
  float4* ztab;        // r-z: FP32 plane tables [nz][nintp]
  double* zc64;        // r-z: FP64 spline rows [nz][nc0], overlaying ztab
  float4* pw32;        // r-z: FP32 z-weights per plane
  double* pw64;        // r-z: FP64 z-weights per plane
  int* pm;             // r-z: first z-coefficient per plane
  uint16_t* cand;      // candidate list
  uint16_t* nodeidx;   // packed node indices
  double* sstep;       // seeded refinement: steps per axis after k quotients
  double* cval;        // FP64 statistic of each candidate (candidate order),
                       // overlaying storage that is dead during the decisions
  float* fscr;         // factored r-z screen: partial sums [group][column][plane][2]
  uint16_t* lanecg;    // factored r-z screen: column | group << 8 per lane
  float* xf;           // XY factored screen: y-collapsed rows [sensor][node row][column]
  float4* xroww;       // XY factored screen: y-weights of each node row
  int* xrowm;          // XY factored screen: first coefficient row of each node row
};
template <int KIND, int NT, bool FA = false, bool FX = false>
__device__ __forceinline__ WaveLds wave_lds(unsigned char* wbase, const DevLrf& L,
                                            const GridP& G) {
  WaveLds w;
  w.recA = (float4*)wbase;
  w.recB = w.recA + L.na;
  w.rec64 = (SensorRec64*)(w.recB + L.na);
  w.ztab = (float4*)(w.rec64 + L.na);
  w.zc64 = (double*)w.ztab;
  int zq = 0, nzp = 0;
  if constexpr (KIND == ANTS_LRF_RZ) {
    const int zt = G.nz * L.nintp, zr = (G.nz * L.nc0 + 1) / 2;
    zq = zt > zr ? zt : zr;
    nzp = G.nz;
  }
  // doubles first, then 4-byte and 2-byte entries (natural alignment)
  w.pw32 = w.ztab + zq;
  w.pw64 = (double*)(w.pw32 + nzp);
  w.sstep = w.pw64 + 4 * nzp;
  const int nxy = G.nx * G.ny;
  const int cplace = cval_place(L.na, G.nz, NT, FA ? nxy : 0);
  w.fscr = (float*)(w.sstep + 3 * kMaxSeedSteps + (cplace == 0 ? 64 * NT : 0));
  w.cval = cplace == 1   ? (double*)w.recA
           : cplace == 2 ? (double*)w.fscr
                         : w.sstep + 3 * kMaxSeedSteps;
  w.pm = (int*)(w.fscr + (FA ? 2 * G.nz * (nxy > 64 ? nxy : 64) : 0));
  w.cand = (uint16_t*)(w.pm + nzp);
  w.nodeidx = w.cand + 64 * NT;
  w.lanecg = w.nodeidx + 64 * NT;
  w.xf = nullptr;
  w.xroww = nullptr;
  w.xrowm = nullptr;
  if constexpr (FX) {
    // after everything else (that size is a multiple of 16 bytes)
    w.xf = (float*)(wbase + wave_lds_bytes(KIND, L.na, G.nz, L.nintp, L.nc0, NT, 0));
    w.xroww = (float4*)(w.xf + kXfFloats);
    w.xrowm = (int*)(w.xroww + 64);
  }
  return w;
}

// Per-wave set-up: node index table and, for seeded refinement, the final
// step divided by the shrink factor k times (iterated quotients), k <
// kMaxSeedSteps, per axis.
template <int KIND, int NT, bool FA = false, bool FX = false>
__device__ __forceinline__ void wave_setup(unsigned char* wbase, const DevLrf& L, const GridP& G,
                                           int lane) {
  const WaveLds w = wave_lds<KIND, NT, FA, FX>(wbase, L, G);
  fill_nodeidx(G, w.nodeidx, 64 * NT, lane);
  if constexpr (FA) {
    // factored screen: lane -> (column of the x-y lattice, sensor group);
    // with more than 64 columns one group and several passes
    const int nxy = G.nx * G.ny;
    const int c = nxy <= 64 ? lane % nxy : lane;
    const int g = nxy <= 64 ? lane / nxy : 0;
    w.lanecg[lane] = (uint16_t)(c | (g << 8));
  }
  if (G.seed_steps && lane < 3) {
    double s = G.sfinal[lane];
    for (int k = 0; k < kMaxSeedSteps; ++k) {
      w.sstep[3 * k + lane] = s;
      s = s / G.shrink;
    }
  }
  wave_sync_lds();
}

template <int KIND>
__device__ __forceinline__ bool make_node(const DevLrf& L, const GridP& G, double cx, double cy,
                                          double cz, double sx, double sy, double sz, int j,
                                          const float4* ztab, const uint16_t* nodeidx,
                                          NodeF<KIND>& nd, double& x, double& y, double& z) {
  const int packed = nodeidx[j];
  const int jx = packed & G.mskx, jy = (packed >> G.shy) & G.msky, jz = packed >> G.shz;
  double ox = (double)(jx - G.hx) * sx;
  double oy = (double)(jy - G.hy) * sy;
  double oz = (double)(jz - G.hz) * sz;
  x = cx + ox;
  y = cy + oy;
  z = cz + oz;
  bool valid = j < G.nn;
  if constexpr (radial_kind(KIND) || KIND == ANTS_LRF_COMPOSITE) {
    nd.ox = (float)(ox * L.inv_d0);
    nd.oy = (float)(oy * L.inv_d0);
  }
  if constexpr (KIND == ANTS_LRF_COMPOSITE) {
    // residual weights; 0 outside its domain (the axial part still counts)
    int m0 = 0, m1 = 0;
    double t0 = 0.0, t1 = 0.0, b0[4], b1[4];
    const bool in = locate64(x, L.xnb0, L.xlo0, L.xhi0, L.xinv_d0, m0, t0) &&
                    locate64(y, L.xnb1, L.xlo1, L.xhi1, L.xinv_d1, m1, t1);
    bweights64(t0, b0);
    bweights64(t1, b1);
    nd.cell = in ? m1 * L.xnc0 + m0 : 0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) nd.w[a * 4 + b] = in ? (float)(b1[a] * b0[b]) : 0.f;
  }
  if constexpr (KIND == ANTS_LRF_SLICED) {
    int m0 = 0, m1 = 0, pz = 0;
    double t0 = 0.0, t1 = 0.0, tz = 0.0, b0[4], b1[4];
    bool in0 = locate64(x, L.nb0, L.lo0, L.hi0, L.inv_d0, m0, t0);
    bool in1 = locate64(y, L.nb1, L.lo1, L.hi1, L.inv_d1, m1, t1);
    bool inz = locate64(z, L.nplanes, L.zlo, L.zhi, L.inv_dz, pz, tz);
    valid = valid && in0 && in1 && inz;
    bweights64(t0, b0);
    bweights64(t1, b1);
    nd.pstride = L.nc0 * L.nc1;
    nd.cell = pz * nd.pstride + m1 * L.nc0 + m0;
    nd.t = (float)tz;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) nd.w[a * 4 + b] = (float)(b1[a] * b0[b]);
  }
  if constexpr (KIND == ANTS_LRF_RZ) {
    int jzc = jz < G.nz ? jz : G.nz - 1;
    nd.tab = ztab + jzc * L.nintp;
    valid = valid && in_domain(z, L.lo1, L.hi1);
  }
  if constexpr (KIND == ANTS_LRF_XY) {
    int m0 = 0, m1 = 0;
    double t0 = 0.0, t1 = 0.0, b0[4], b1[4];
    bool in0 = locate64(x, L.nb0, L.lo0, L.hi0, L.inv_d0, m0, t0);
    bool in1 = locate64(y, L.nb1, L.lo1, L.hi1, L.inv_d1, m1, t1);
    valid = valid && in0 && in1;
    bweights64(t0, b0);
    bweights64(t1, b1);
    nd.cell = m1 * L.nc0 + m0;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) nd.w[a * 4 + b] = (float)(b1[a] * b0[b]);
  }
  return valid;
}

// exp(s / 2) of a seed's log-variance, once per event: kept out of line so
// that the exponential's constants are not held in registers (and spilled)
// across the event loop
__device__ __attribute__((noinline)) double seed_sigma(double s) { return exp(0.5 * s); }

// log2(1 + x) with small relative error for small |x| (per node only)
__device__ __forceinline__ float log2_1p(float x) {
  float u = 1.0f + x;
  float d = u - 1.0f;
  return d == 0.0f ? x * kLog2e : __builtin_amdgcn_logf(u) * (x / d);
}

// --------------------------------------------------------------- kernel

// Where process_event reads its parameters.  KargSrc re-reads the kernel's
// parameter block (scalar loads) at each event, iteration and output stage
// instead of holding it in scalar registers for the whole launch: the block
// exceeds the register budget, and spilling it costs VALU lane moves.
struct ParView {
  const DevLrf& L;
  const GridP& G;
  const IoP& io;
};
struct KArgs {
  DevLrf L;
  GridP G;
  IoP io;
  int64_t waves_total;
  int per_wave_bytes, btab_n;
};
typedef const __attribute__((address_space(4))) KArgs KArgsK;
// the launch's own kernel arguments (constant memory)
struct KargSrc {
  KArgsK* kp;
  __device__ __forceinline__ ParView view() const {
    KArgsK* p = kp;
    asm volatile("" : "+s"(p));
    const KArgs& a = *(const KArgs*)p;
    return {a.L, a.G, a.io};
  }
};
// parameters already in registers or memory chosen by the caller
struct RefSrc {
  const DevLrf& L;
  const GridP& G;
  const IoP& io;
  __device__ __forceinline__ ParView view() const { return {L, G, io}; }
};

// One event on one wavefront.  btab: block-shared tables (LDS); wbase: this
// wave's LDS region (sensor records, r-z plane tables, candidate list).
template <int KIND, int STAT, int NT, int SL, bool NN, int FZ, class Src>
__device__ __forceinline__ void process_event(const Src& src, const int64_t e,
                                              const float4* btab, unsigned char* wbase,
                                              const int lane) {
  // FZ > 0: r-z, the column-factored screen over FZ z-planes; XY, the
  // screen from y-collapsed coefficient rows staged in LDS
  constexpr bool FA = FZ > 0 && KIND == ANTS_LRF_RZ;
  constexpr bool FX = FZ > 0 && KIND == ANTS_LRF_XY;
  const ParView V0 = src.view();
  const DevLrf& L = V0.L;
  const GridP& G = V0.G;
  const IoP& io = V0.io;
  const WaveLds W = wave_lds<KIND, NT, FA, FX>(wbase, L, G);
  float4* recA = W.recA;
  float4* recB = W.recB;
  SensorRec64* rec64 = W.rec64;
  float4* ztab = W.ztab;
  uint16_t* cand = W.cand;
  const uint16_t* nodeidx = W.nodeidx;
  // r-z: FP64 spline rows collapsed on each z-plane of the current grid
  // (they overlay the FP32 plane tables, which the FP64 decision does not
  // read), the z-weights and the first z-coefficient of each plane
  double* zc64 = W.zc64;
  double* pw64 = W.pw64;
  int* pm64 = W.pm;
  const int na = L.na;
  const int nlast = L.nintp - 1;
  const float finv = L.finv0;
  const float flf = (float)G.lfloor;
  const float fvf = (float)G.vfloor;
  const float* row = io.sig + e * io.ld;

  // ---------------- event set-up: signals of the active sensors
  float nq[SL];
  int posq[SL];
  double N = 0.0, cw = 0.0, cxs = 0.0, cys = 0.0;
  bool bad = false;
  float best_n = -1.0f;
  int best_a = 1 << 30;
  // the centroid is needed only for the centroid start
  const bool cog = !(G.start == ANTS_START_SEED && io.seeds) && G.start != ANTS_START_MAXSENSOR;
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    int a = lane + 64 * q;
    nq[q] = 0.f;
    if (a < na) {
      float n = row[L.col[a]];
      nq[q] = n;
      if (!(n >= 0.f) || !(n < kInf)) {
        bad = true;
      } else {
        N += (double)n;
        if (cog) {
          double wgt = (double)n / L.g[a];
          cw += wgt;
          cxs += L.X[a] * wgt;
          cys += L.Y[a] * wgt;
        }
        if (n > best_n) { best_n = n; best_a = a; }
      }
    }
  }
  bool any_bad = __ballot(bad) != 0ull;
  N = uni(wsum_d(N));
  int ndf = na - (G.dim + 1);
  int status = 0;
  if (na == 0) status = ANTS_EV_NO_ACTIVE;
  else if (any_bad) status = ANTS_EV_BAD_INPUT;
  else if (!(N > 0.0)) status = ANTS_EV_EMPTY;
  if (status) {
    if (lane == 0) {
      float nan = __builtin_nanf("");
      io.x[e] = nan; io.y[e] = nan; io.z[e] = nan; io.E[e] = nan;
      io.lnl[e] = nan; io.chi2[e] = nan; io.ndf[e] = ndf; io.status[e] = status;
      if (io.nfp) io.nfp[e] = 0;
    }
    if (io.path && lane < G.K) io.path[e * G.K + lane] = -1;
    return;
  }
  if (cog) {
    cw = wsum_d(cw);
    cxs = wsum_d(cxs);
    cys = wsum_d(cys);
  }

  double cx, cy, cz = G.z_start;
  if (G.start == ANTS_START_SEED && io.seeds) {
    cx = io.seeds[e * 4 + 0];
    cy = io.seeds[e * 4 + 1];
    if (G.dim == 3) cz = io.seeds[e * 4 + 2];
  } else if (G.start == ANTS_START_MAXSENSOR) {
    wargmax_f(best_n, best_a);
    best_a = uni(best_a);
    cx = L.X[best_a];
    cy = L.Y[best_a];
  } else {
    cx = cxs / cw;
    cy = cys / cw;
  }
  cx = uni(cx);
  cy = uni(cy);
  cz = uni(cz);

  // sensor cuts: sensors with a signal below cut_signal or farther (x-y)
  // than cut_dist from the start are passive for the rest of the event
  bool ign[SL];
  int na_ev = na;
#pragma unroll
  for (int q = 0; q < SL; ++q) ign[q] = false;
  if (G.cut_signal > 0.0 || G.cut_dist > 0.0) {
    double Nk = 0.0;
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      const int a = lane + 64 * q;
      if (a < na) {
        bool ig = G.cut_signal > 0.0 && (double)nq[q] < G.cut_signal;
        if (G.cut_dist > 0.0) {
          const double dx = L.X[a] - cx, dy = L.Y[a] - cy;
          ig = ig || sqrt(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy))) > G.cut_dist;
        }
        ign[q] = ig;
        if (!ig) Nk += (double)nq[q];
      }
    }
    int nk = 0;
#pragma unroll
    for (int q = 0; q < SL; ++q) nk += __popcll(__ballot(lane + 64 * q < na && !ign[q]));
    N = uni(wsum_d(Nk));
    na_ev = nk;
    ndf = nk - (G.dim + 1);
    const int st = nk == 0 ? ANTS_EV_NO_ACTIVE : !(N > 0.0) ? ANTS_EV_EMPTY : 0;
    if (st) {
      if (lane == 0) {
        float nan = __builtin_nanf("");
        io.x[e] = nan; io.y[e] = nan; io.z[e] = nan; io.E[e] = nan;
        io.lnl[e] = nan; io.chi2[e] = nan; io.ndf[e] = ndf; io.status[e] = st | G.or_status;
        if (io.nfp) io.nfp[e] = 0;
      }
      if (io.path && lane < G.K) io.path[e * G.K + lane] = -1;
      return;
    }
  }

  // record positions with counted sensors first, then silent ones, then the
  // ignored (the order of every iteration in which no sensor reaches the end
  // of the LRF domain)
  int posq0[SL], npos0 = 0;
  {
    uint64_t mpos[SL], mzero[SL], mign[SL];
    int nzero = 0;
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      const int a = lane + 64 * q;
      mpos[q] = __ballot(a < na && !ign[q] && nq[q] > 0.f);
      mzero[q] = __ballot(a < na && !ign[q] && !(nq[q] > 0.f));
      mign[q] = __ballot(a < na && ign[q]);
      npos0 += __popcll(mpos[q]);
      nzero += __popcll(mzero[q]);
    }
    int bp = 0, bz = npos0, bi = npos0 + nzero;
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      posq0[q] = ign[q] ? bi + prefix_count(mign[q])
                 : nq[q] > 0.f ? bp + prefix_count(mpos[q]) : bz + prefix_count(mzero[q]);
      bp += __popcll(mpos[q]);
      bz += __popcll(mzero[q]);
      bi += __popcll(mign[q]);
    }
  }
  // FP64 sensor records in sensor order; FP32 table offsets in registers
  const float N32 = (float)N;
  int tofq[SL];
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int a = lane + 64 * q;
    tofq[q] = 0;
    if (a < na) {
      SensorRec64 r;
      r.X = L.X[a];
      r.Y = L.Y[a];
      r.g = L.g[a];
      r.coff = coef_off64<KIND>(L, a);
      r.n = ign[q] ? -1.0f : nq[q];   // negative: ignored by the cuts
      rec64[a] = r;
      tofq[q] = KIND == ANTS_LRF_XY          ? L.tab[a] * L.nc0 * L.nc1
                : KIND == ANTS_LRF_SLICED    ? L.tab[a] * L.nplanes * L.nc0 * L.nc1
                : KIND == ANTS_LRF_COMPOSITE ? L.xtab[a] * L.xnc0 * L.xnc1
                                             : L.tab[a] * L.nintp;
    }
  }

  double sx = G.s0x, sy = G.s0y, sz = G.s0z;
  int Kev = G.K;
  if (G.seed_steps && io.seeds) {
    // steps from the seed's predicted spread: the smallest iteration count
    // in [kmin, kmax] whose first step covers kappa * sigma on every axis,
    // ending on the configured final step
    const double lv = io.seeds[e * 4 + 3];
    const double sg = uni(seed_sigma(lv) * G.kappa);
    const double* st = W.sstep;
    int kk = G.kmin - 1;
    if (!(sg < __builtin_huge_val())) {
      kk = G.kmax - 1;
    } else {
      for (; kk < G.kmax - 1; ++kk) {
        const bool short_ = (G.nx > 1 && st[3 * kk] < sg * G.sscale[0]) ||
                            (G.ny > 1 && st[3 * kk + 1] < sg * G.sscale[1]) ||
                            (G.nz > 1 && st[3 * kk + 2] < sg * G.sscale[2]);
        if (!short_) break;
      }
    }
    kk = uni(kk);
    Kev = kk + 1;
    sx = uni(G.nx > 1 ? st[3 * kk] : 0.0);
    sy = uni(G.ny > 1 ? st[3 * kk + 1] : 0.0);
    sz = uni(G.nz > 1 ? st[3 * kk + 2] : 0.0);
  }
  int nfp = 0;
  // LRF values at the previous iteration's best screened node: the next
  // centre is that node or a near-tie neighbour, so they serve as the next
  // iteration's reference values (the centre-relative form is exact for any
  // reference; its rounding only needs the reference near the nodes)
  float Lprev[SL];
  bool have_prev = false;
#pragma unroll
  for (int q = 0; q < SL; ++q) Lprev[q] = 0.f;
  for (int k = 0; k < Kev; ++k) {
    const int lk = opaque(lane);
    const ParView Vk = src.view();
    const DevLrf& L = Vk.L;
    const GridP& G = Vk.G;
    const IoP& io = Vk.io;
    // ---- r-z: collapse the table along z for this iteration's planes
    if constexpr (KIND == ANTS_LRF_RZ) {
      // plane weights once per plane
      float4* pw = W.pw32;
      int* pm = W.pm;
      for (int jz = lane; jz < G.nz; jz += 64) {
        const double zz = cz + (double)(jz - G.hz) * sz;
        int mz;
        double tz, bz[4];
        if (locate64(zz, L.nb1, L.lo1, L.hi1, L.inv_d1, mz, tz)) {
          bweights64(tz, bz);
        } else {
          bz[0] = bz[1] = bz[2] = bz[3] = 0.0;
          mz = 0;
        }
        pw[jz] = make_float4((float)bz[0], (float)bz[1], (float)bz[2], (float)bz[3]);
        pm[jz] = mz;
        for (int r = 0; r < 4; ++r) pw64[4 * jz + r] = bz[r];
      }
      wave_sync_lds();
      const int ntot = G.nz * L.nintp;
      const float inv_nintp = 1.0f / (float)L.nintp;
      for (int i = lane; i < ntot; i += 64) {
        const int jz = (int)(((float)i + 0.5f) * inv_nintp);
        const int m = i - jz * L.nintp;
        const float4 w = pw[jz];
        const float4* P = btab + pm[jz] * L.nintp + m;
        const float4 P0 = P[0], P1 = P[L.nintp], P2 = P[2 * L.nintp], P3 = P[3 * L.nintp];
        float4 acc;
        acc.x = fmaf(w.w, P3.x, fmaf(w.z, P2.x, fmaf(w.y, P1.x, w.x * P0.x)));
        acc.y = fmaf(w.w, P3.y, fmaf(w.z, P2.y, fmaf(w.y, P1.y, w.x * P0.y)));
        acc.z = fmaf(w.w, P3.z, fmaf(w.z, P2.z, fmaf(w.y, P1.z, w.x * P0.z)));
        acc.w = fmaf(w.w, P3.w, fmaf(w.z, P2.w, fmaf(w.y, P1.w, w.x * P0.w)));
        ztab[i] = acc;
      }
      wave_sync_lds();
    }
    // r-z: FP64 rows of the planes, made on the first FP64 decision of the
    // iteration (most iterations decide from the screen alone)
    auto make_rows = [&]() {
      if constexpr (KIND == ANTS_LRF_RZ) {
        const int nct = G.nz * L.nc0;
        const float inv_nc0 = 1.0f / (float)L.nc0;
        for (int i = lane; i < nct; i += 64) {
          const int jz = (int)(((float)i + 0.5f) * inv_nc0);
          const int c = i - jz * L.nc0;
          const double* col = L.c64 + (size_t)pm64[jz] * L.nc0 + c;
          const double* w = pw64 + 4 * jz;
          zc64[i] = w[0] * col[0] + w[1] * col[L.nc0] + w[2] * col[2 * L.nc0] +
                    w[3] * col[3 * L.nc0];
        }
        wave_sync_lds();
      }
    };

    // ---- reference at the centre, per sensor (lane-parallel)
    NodeF<KIND> ndc;
    if (!have_prev) {
      double xx, yy, zz;
      int jc = (G.hz * G.ny + G.hy) * G.nx + G.hx;
      make_node<KIND>(L, G, cx, cy, cz, sx, sy, sz, jc, ztab, nodeidx, ndc, xx, yy, zz);
    }
    // ---- reference values at the centre and order of the FP32 records for
    // this iteration.  Radial kinds: the LRF jumps to zero at the end of its
    // domain, where the FP32 and FP64 distances may fall on different sides.
    // A sensor below the end at every node of the grid (with a band for the
    // FP32 distance error) is "inside"; one beyond it at every node has a
    // zero LRF in both precisions and terms equal at every node, so the
    // screen skips it; any other is an "edge" sensor, screened by loops of
    // their own that send the nodes within the band to FP64.  Order: counted
    // inside, counted edge, zero-signal inside, zero-signal edge, beyond.
    const float vhi = (float)nlast;   // end of the domain, in breakpoint spacings
    float band = 0.f;
    float Sc = 0.f;
    float dXq[SL], dYq[SL], Lcq[SL];
    float ex = 0.f, ey = 0.f, lo2 = 0.f, hi2 = 0.f;
    bool reach = false;   // some sensor may reach the end of the domain
    if constexpr (radial_kind(KIND)) {
      ex = (float)((double)(G.nx - 1 - G.hx) * sx * L.inv_d0);
      ey = (float)((double)(G.ny - 1 - G.hy) * sy * L.inv_d0);
      band = 4e-6f * (vhi + 2.f * (ex + ey) + 1.f);
      lo2 = (vhi - band) * (vhi - band);
      hi2 = (vhi + band) * (vhi + band);
    }
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      const int a = lane + 64 * q;
      dXq[q] = dYq[q] = Lcq[q] = 0.f;
      if (a < na) {
        const SensorRec64 r = rec64[a];
        const float dX = (float)((r.X - cx) * L.inv_d0), dY = (float)((r.Y - cy) * L.inv_d0);
        const float Lc = have_prev ? Lprev[q]
                                   : lrf32<KIND, NN>(ndc, dX, dY, tofq[q], btab, scr_c32<KIND>(L), scr_nc0<KIND>(L),
                                                     finv, nlast);
        if (!ign[q]) Sc = fmaf((float)r.g, Lc, Sc);
        dXq[q] = dX;
        dYq[q] = dY;
        Lcq[q] = Lc;
        if constexpr (radial_kind(KIND)) {
          const float fx = fabsf(dX) + ex, fy = fabsf(dY) + ey;
          reach = reach || (!ign[q] && !(fmaf(fx, fx, fy * fy) < lo2));
        }
      }
    }
    Sc = uni(wsum_f(Sc));
    const bool rel = Sc > 0.f;   // centre-relative form available
    int n_ci = npos0, n_pos = npos0, z_end = na_ev, n_scr = na_ev;
    if (__ballot(reach) == 0ull) {
#pragma unroll
      for (int q = 0; q < SL; ++q) posq[q] = posq0[q];
    } else {
      // categories: 0 counted inside, 1 counted edge, 2 zero-signal inside,
      // 3 zero-signal edge, 4 beyond
      int key[SL];
#pragma unroll
      for (int q = 0; q < SL; ++q) {
        const float ax = fabsf(dXq[q]), ay = fabsf(dYq[q]);
        const float nx0 = fmaxf(ax - ex, 0.f), ny0 = fmaxf(ay - ey, 0.f);
        const float fx = ax + ex, fy = ay + ey;
        const int cls = fmaf(fx, fx, fy * fy) < lo2 ? 0 : fmaf(nx0, nx0, ny0 * ny0) > hi2 ? 2 : 1;
        key[q] = (cls == 2 || ign[q]) ? 4 : (nq[q] > 0.f ? 0 : 2) + cls;
      }
      uint64_t mk[SL][5];
      int cnt[5] = {0, 0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < SL; ++q) {
        const int a = lane + 64 * q;
        const bool in = a < na;
        const uint64_t mv = __ballot(in), mc = __ballot(in && (key[q] == 0 || key[q] == 1));
        const uint64_t me = __ballot(in && (key[q] == 1 || key[q] == 3));
        const uint64_t mb = __ballot(in && key[q] == 4);
        mk[q][0] = mc & ~me;
        mk[q][1] = mc & me;
        mk[q][2] = mv & ~mc & ~me & ~mb;
        mk[q][3] = mv & ~mc & me;
        mk[q][4] = mb;
#pragma unroll
        for (int c = 0; c < 5; ++c) cnt[c] += __popcll(mk[q][c]);
      }
      int run[5];
      run[0] = 0;
#pragma unroll
      for (int c = 1; c < 5; ++c) run[c] = run[c - 1] + cnt[c - 1];
      n_ci = run[1];
      n_pos = run[2];
      z_end = run[3];
      n_scr = run[4];
#pragma unroll
      for (int q = 0; q < SL; ++q) {
        int pos = 0;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          if (key[q] == c) pos = run[c] + prefix_count(mk[q][c]);
          run[c] += __popcll(mk[q][c]);
        }
        posq[q] = pos;
      }
    }
    // absolute form (no centre reference): L_c = 0 and 1/L_c = 1 make dS = S
    // and the log terms absolute
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      const int a = lane + 64 * q;
      if (a < na) {
        const float Lc = rel ? Lcq[q] : 0.f;
        recA[posq[q]] = make_float4(dXq[q], dYq[q], nq[q], rel ? 1.0f / fmaxf(Lc, flf) : 1.f);
        recB[posq[q]] = make_float4((float)rec64[a].g, Lc, __int_as_float(tofq[q]),
                                    __int_as_float(a));
      }
    }
    const float iSc = rel ? 1.0f / Sc : 1.0f;
    wave_sync_lds();

    // ---- node set-up
    // grids of at most 32 nodes split the sensors between the two halves of
    // the wave: lanes l and l + 32 both hold node l, each sums over every
    // other sensor, and the halves add their sums
    const bool split = !FA && !FX && NT == 1 && G.nn <= 32;
    // with several tiles and at most 32 nodes in the last one (ML screen),
    // only the last tile is split that way
    const bool lsplit =
        !FA && !FX && STAT == ANTS_STAT_ML && NT >= 2 && G.nn - 64 * (NT - 1) <= 32;
    const int hb = (split || lsplit) ? (lk >> 5) : 0;
    const int pstep = split ? 2 : 1;
    NodeF<KIND> nd[NT];
    bool valid[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      double xx, yy, zz;
      const bool half = split || (lsplit && t == NT - 1);
      const int j = t * 64 + (half ? (lk & 31) : lk);
      valid[t] = make_node<KIND>(L, G, cx, cy, cz, sx, sy, sz, j, ztab, nodeidx, nd[t], xx, yy, zz);
      if (half) valid[t] = valid[t] && lk < 32;
    }
    // XY factored screen.  Every sensor's bicubic is on the same knot grid,
    // so a node's x-weights and first coefficient column depend on its
    // column only and its y-weights and first row on its row only.  Each
    // sensor's coefficients are collapsed along y once per node row (over
    // the columns the grid touches) and staged in LDS; a node then reads 4
    // values and applies its 4 x-weights.  Here: the x-weights and offset of
    // each node, and the y-weights and first row of each node row.
    float4 xw[NT];
    int xoff[NT];
    int xm0 = 0, xwc = 4;
    if constexpr (FX) {
      int m0t[NT], jyt[NT];
      int mlo = 1 << 30, mhi = -1;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const int j = t * 64 + lk;
        const int pk = nodeidx[j];
        const int jx = pk & G.mskx, jy = (pk >> G.shy) & G.msky;
        const double x = cx + (double)(jx - G.hx) * sx;
        const double y = cy + (double)(jy - G.hy) * sy;
        int m0 = 0, m1 = 0;
        double t0 = 0.0, t1 = 0.0, b0[4];
        const bool inx = locate64(x, L.nb0, L.lo0, L.hi0, L.inv_d0, m0, t0);
        const bool iny = locate64(y, L.nb1, L.lo1, L.hi1, L.inv_d1, m1, t1);
        bweights64(t0, b0);
        xw[t] = make_float4((float)b0[0], (float)b0[1], (float)b0[2], (float)b0[3]);
        m0t[t] = inx ? m0 : -1;
        jyt[t] = jy;
        if (j < G.nn && inx) {
          mlo = m0 < mlo ? m0 : mlo;
          mhi = m0 > mhi ? m0 : mhi;
        }
        if (j < G.nn && jx == 0) {
          double b1[4];
          bweights64(t1, b1);
          W.xroww[jy] = make_float4((float)b1[0], (float)b1[1], (float)b1[2], (float)b1[3]);
          W.xrowm[jy] = iny ? m1 : 0;
        }
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const int a = __shfl_xor(mlo, o), b = __shfl_xor(mhi, o);
        mlo = a < mlo ? a : mlo;
        mhi = b > mhi ? b : mhi;
      }
      mlo = uni(mlo);
      mhi = uni(mhi);
      if (mhi < 0) mlo = mhi = 0;   // no node column inside the domain
      xm0 = mlo;
      xwc = mhi - mlo + 4;
      // columns outside the domain (invalid nodes) read the first column
#pragma unroll
      for (int t = 0; t < NT; ++t) xoff[t] = jyt[t] * xwc + (m0t[t] >= 0 ? m0t[t] - xm0 : 0);
      wave_sync_lds();
    }
    const int xstride = G.ny * xwc;   // floats per staged sensor
    const int xcap = FX ? uni(kXfFloats / xstride) : 1;   // sensors per chunk (>= 1)
    const float xinv_wc = FX ? 1.0f / (float)xwc : 1.0f;
    // stage records [p0, p0 + cnt): row jy of sensor p at p * xstride + jy *
    // xwc; lanes take (sensor, column), node rows go in threes with their
    // 12 loads issued together
    auto xf_stage = [&](int p0, int cnt) {
      if constexpr (FX) {
        const int total = cnt * xwc;
        const int nc0 = L.nc0, ny = G.ny;
        for (int i = lk; i < total; i += 64) {
          const int pp = (int)(((float)i + 0.5f) * xinv_wc);
          const int col = i - pp * xwc;
          const float* src = L.c32 + __float_as_int(recB[p0 + pp].z) + xm0 + col;
          float* dst = W.xf + pp * xstride + col;
          for (int jy0 = 0; jy0 < ny; jy0 += 3) {
            float4 w[3];
            float c[3][4];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
              const int jy = jy0 + u < ny ? jy0 + u : ny - 1;   // in bounds; not stored
              w[u] = W.xroww[jy];
              const float* q = src + W.xrowm[jy] * nc0;
#pragma unroll
              for (int a = 0; a < 4; ++a) c[u][a] = q[a * nc0];
            }
#pragma unroll
            for (int u = 0; u < 3; ++u)
              if (jy0 + u < ny)
                dst[(jy0 + u) * xwc] =
                    fmaf(w[u].w, c[u][3], fmaf(w[u].z, c[u][2], fmaf(w[u].y, c[u][1], w[u].x * c[u][0])));
          }
        }
        wave_sync_lds();
      }
    };
    // LRF of node tile t from sensor p's staged rows (base at chunk record p0)
    auto xf_lrf = [&](const float* rows, int t) -> float {
      const float* r = rows + xoff[t];
      return fmaxf(fmaf(xw[t].w, r[3], fmaf(xw[t].z, r[2], fmaf(xw[t].y, r[1], xw[t].x * r[0]))),
                   0.f);
    };

    // ---- FP32 screen
    float D[NT], Snode[NT];
    if constexpr (STAT == ANTS_STAT_ML) {
      float dS[NT], T[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) { dS[t] = 0.f; T[t] = 0.f; }
      if constexpr (FX) {
        // chunks of staged sensors; XY has no edge classes: counted sensors
        // are [0, n_ci), zero-signal ones [n_pos, z_end)
        for (int p0 = 0; p0 < z_end; p0 += xcap) {
          const int p1 = p0 + xcap < z_end ? p0 + xcap : z_end;
          xf_stage(p0, p1 - p0);
          const int pc = p1 < n_ci ? p1 : n_ci;
#pragma unroll 2
          for (int p = p0; p < pc; ++p) {
            const float4 A = recA[p], B = recB[p];
            const float* rows = W.xf + (p - p0) * xstride;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              const float Lv = xf_lrf(rows, t);
              dS[t] = fmaf(B.x, Lv - B.y, dS[t]);
              T[t] = fmaf(A.z, __builtin_amdgcn_logf(Lv * A.w), T[t]);
            }
          }
#pragma unroll 2
          for (int p = p0 > n_pos ? p0 : n_pos; p < p1; ++p) {
            const float4 B = recB[p];
            const float* rows = W.xf + (p - p0) * xstride;
#pragma unroll
            for (int t = 0; t < NT; ++t) dS[t] = fmaf(B.x, xf_lrf(rows, t) - B.y, dS[t]);
          }
          wave_sync_lds();
        }
      } else if constexpr (FA) {
        // r-z, 2 to 8 z-planes: the distance from a sensor depends on the
        // node's x-y column only, so lanes take (column, sensor group) and
        // evaluate every plane from one distance; the groups' partial sums
        // are then added per node through LDS
        const int nxy = G.nx * G.ny;
        constexpr int nz = FZ;   // equals G.nz
        const int lcg = W.lanecg[lk];
        const int c0 = lcg & 255, grp = lcg >> 8;
        const int ngrp = nxy <= 64 ? 64 / nxy : 1;
        float* scr = W.fscr;
        for (int cbase = 0; cbase < nxy; cbase += 64) {
          const int c = c0 + cbase;
          if (c < nxy && grp < ngrp) {
            const int pk = nodeidx[c];   // node c: column c on the first plane
            const int jx = pk & G.mskx, jy = (pk >> G.shy) & G.msky;
            const float ox = (float)((double)(jx - G.hx) * sx * L.inv_d0);
            const float oy = (float)((double)(jy - G.hy) * sy * L.inv_d0);
            float aS[nz], aT[nz];
#pragma unroll
            for (int q = 0; q < nz; ++q) { aS[q] = 0.f; aT[q] = 0.f; }
            const int pstride = L.nintp;
            for (int p = grp; p < n_ci; p += ngrp) {
              const float4 A = recA[p], B = recB[p];
              const float dx = ox - A.x, dy = oy - A.y;
              const float v = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
              const int m = (int)fminf(v, (float)nlast);
              const float tt = __builtin_amdgcn_fractf(v);
              const float4* tp = ztab + m;
              float4 cf[nz];
#pragma unroll
              for (int q = 0; q < nz; ++q) cf[q] = tp[q * pstride];
#pragma unroll
              for (int q = 0; q < nz; ++q) {
                float Lv = fmaf(fmaf(fmaf(cf[q].w, tt, cf[q].z), tt, cf[q].y), tt, cf[q].x);
                if (!NN) Lv = fmaxf(Lv, 0.f);
                aS[q] = fmaf(B.x, Lv - B.y, aS[q]);
                aT[q] = fmaf(A.z, __builtin_amdgcn_logf(Lv * A.w), aT[q]);
              }
            }
            for (int p = n_pos + grp; p < z_end; p += ngrp) {
              const float4 A = recA[p], B = recB[p];
              const float dx = ox - A.x, dy = oy - A.y;
              const float v = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
              const int m = (int)fminf(v, (float)nlast);
              const float tt = __builtin_amdgcn_fractf(v);
              const float4* tp = ztab + m;
              float4 cf[nz];
#pragma unroll
              for (int q = 0; q < nz; ++q) cf[q] = tp[q * pstride];
#pragma unroll
              for (int q = 0; q < nz; ++q) {
                float Lv = fmaf(fmaf(fmaf(cf[q].w, tt, cf[q].z), tt, cf[q].y), tt, cf[q].x);
                if (!NN) Lv = fmaxf(Lv, 0.f);
                aS[q] = fmaf(B.x, Lv - B.y, aS[q]);
              }
            }
            // edge sensors: a column within the band of the domain end makes
            // its nodes non-finite (FP64); beyond the end the LRF is zero and
            // the logarithm takes the floor, as in FP64
            bool kn = false;
            for (int p = n_ci + grp; p < n_pos; p += ngrp) {
              const float4 A = recA[p], B = recB[p];
              const float dx = ox - A.x, dy = oy - A.y;
              const float v = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
              const int m = (int)fminf(v, (float)nlast);
              const float tt = __builtin_amdgcn_fractf(v);
              const float4* tp = ztab + m;
              kn = kn || fabsf(v - vhi) < band;
              const float fwb = v >= vhi ? flf * A.w : 0.f;
#pragma unroll
              for (int q = 0; q < nz; ++q) {
                const float4 cq = tp[q * pstride];
                float Lv = fmaf(fmaf(fmaf(cq.w, tt, cq.z), tt, cq.y), tt, cq.x);
                if (!NN) Lv = fmaxf(Lv, 0.f);
                aS[q] = fmaf(B.x, Lv - B.y, aS[q]);
                aT[q] = fmaf(A.z, __builtin_amdgcn_logf(fmaxf(Lv * A.w, fwb)), aT[q]);
              }
            }
            for (int p = z_end + grp; p < n_scr; p += ngrp) {
              const float4 A = recA[p], B = recB[p];
              const float dx = ox - A.x, dy = oy - A.y;
              const float v = __builtin_amdgcn_sqrtf(fmaf(dx, dx, dy * dy));
              const int m = (int)fminf(v, (float)nlast);
              const float tt = __builtin_amdgcn_fractf(v);
              const float4* tp = ztab + m;
              kn = kn || fabsf(v - vhi) < band;
#pragma unroll
              for (int q = 0; q < nz; ++q) {
                const float4 cq = tp[q * pstride];
                float Lv = fmaf(fmaf(fmaf(cq.w, tt, cq.z), tt, cq.y), tt, cq.x);
                if (!NN) Lv = fmaxf(Lv, 0.f);
                aS[q] = fmaf(B.x, Lv - B.y, aS[q]);
              }
            }
            float* o = scr + (grp * nxy + c) * nz * 2;
#pragma unroll
            for (int q = 0; q < nz; ++q) {
              o[2 * q] = aS[q];
              o[2 * q + 1] = kn ? __builtin_nanf("") : aT[q];
            }
          }
        }
        wave_sync_lds();
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const int j = t * 64 + lk;
          if (j < G.nn) {
            const int pk = nodeidx[j];
            const int c = ((pk >> G.shy) & G.msky) * G.nx + (pk & G.mskx);
            const float* o = scr + (c * nz + (pk >> G.shz)) * 2;
            float a = 0.f, b = 0.f;
            for (int g = 0; g < ngrp; ++g) {
              a += o[g * nxy * nz * 2];
              b += o[g * nxy * nz * 2 + 1];
            }
            dS[t] = a;
            T[t] = b;
          }
        }
      } else if (lsplit) {
        // full tiles take sensors p and p + 1, the last tile's half-waves
        // one each
        constexpr int LT = NT - 1;
        int p = 0;
        for (; p + 2 <= n_ci; p += 2) {
          const float4 A0 = recA[p], B0 = recB[p], A1 = recA[p + 1], B1 = recB[p + 1];
          const float4 Ah = recA[p + hb], Bh = recB[p + hb];
          const int o0 = __float_as_int(B0.z), o1 = __float_as_int(B1.z), oh = __float_as_int(Bh.z);
#pragma unroll
          for (int t = 0; t < LT; ++t) {
            const float L0 = lrf32<KIND, NN>(nd[t], A0.x, A0.y, o0, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
            dS[t] = fmaf(B0.x, L0 - B0.y, dS[t]);
            T[t] = fmaf(A0.z, __builtin_amdgcn_logf(L0 * A0.w), T[t]);
            const float L1 = lrf32<KIND, NN>(nd[t], A1.x, A1.y, o1, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
            dS[t] = fmaf(B1.x, L1 - B1.y, dS[t]);
            T[t] = fmaf(A1.z, __builtin_amdgcn_logf(L1 * A1.w), T[t]);
          }
          const float Lh = lrf32<KIND, NN>(nd[LT], Ah.x, Ah.y, oh, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
          dS[LT] = fmaf(Bh.x, Lh - Bh.y, dS[LT]);
          T[LT] = fmaf(Ah.z, __builtin_amdgcn_logf(Lh * Ah.w), T[LT]);
        }
        if (p < n_ci) {
          const float4 A = recA[p], B = recB[p];
          const int o = __float_as_int(B.z);
#pragma unroll
          for (int t = 0; t < LT; ++t) {
            const float Lv = lrf32<KIND, NN>(nd[t], A.x, A.y, o, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
            dS[t] = fmaf(B.x, Lv - B.y, dS[t]);
            T[t] = fmaf(A.z, __builtin_amdgcn_logf(Lv * A.w), T[t]);
          }
          const float w = hb ? 0.f : 1.f;
          const float Lh = lrf32<KIND, NN>(nd[LT], A.x, A.y, o, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
          dS[LT] = fmaf(B.x * w, Lh - B.y, dS[LT]);
          T[LT] = fmaf(A.z * w, __builtin_amdgcn_logf(Lh * A.w), T[LT]);
        }
        for (p = n_pos; p + 2 <= z_end; p += 2) {
          const float4 A0 = recA[p], B0 = recB[p], A1 = recA[p + 1], B1 = recB[p + 1];
          const float4 Ah = recA[p + hb], Bh = recB[p + hb];
          const int o0 = __float_as_int(B0.z), o1 = __float_as_int(B1.z), oh = __float_as_int(Bh.z);
#pragma unroll
          for (int t = 0; t < LT; ++t) {
            const float L0 = lrf32<KIND, NN>(nd[t], A0.x, A0.y, o0, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
            dS[t] = fmaf(B0.x, L0 - B0.y, dS[t]);
            const float L1 = lrf32<KIND, NN>(nd[t], A1.x, A1.y, o1, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
            dS[t] = fmaf(B1.x, L1 - B1.y, dS[t]);
          }
          const float Lh = lrf32<KIND, NN>(nd[LT], Ah.x, Ah.y, oh, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
          dS[LT] = fmaf(Bh.x, Lh - Bh.y, dS[LT]);
        }
        if (p < z_end) {
          const float4 A = recA[p], B = recB[p];
          const int o = __float_as_int(B.z);
#pragma unroll
          for (int t = 0; t < LT; ++t) {
            const float Lv = lrf32<KIND, NN>(nd[t], A.x, A.y, o, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
            dS[t] = fmaf(B.x, Lv - B.y, dS[t]);
          }
          const float Lh = lrf32<KIND, NN>(nd[LT], A.x, A.y, o, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
          dS[LT] = fmaf(hb ? 0.f : B.x, Lh - B.y, dS[LT]);
        }
        dS[LT] += __shfl_xor(dS[LT], 32);
        T[LT] += __shfl_xor(T[LT], 32);
      } else {
        int p = 0;
        for (; p + pstep <= n_ci; p += pstep) {
          float4 A = recA[p + hb], B = recB[p + hb];
          int tofs = __float_as_int(B.z);
  #pragma unroll
          for (int t = 0; t < NT; ++t) {
            float Lv = lrf32<KIND, NN>(nd[t], A.x, A.y, tofs, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
            dS[t] = fmaf(B.x, Lv - B.y, dS[t]);
            T[t] = fmaf(A.z, __builtin_amdgcn_logf(Lv * A.w), T[t]);
          }
        }
        if (split && p < n_ci) {
          // odd count: the first half takes the last sensor, the second adds
          // zero (or NaN where the first half's term is infinite already)
          float4 A = recA[p], B = recB[p];
          const float w = hb ? 0.f : 1.f;
          float Lv = lrf32<KIND, NN>(nd[0], A.x, A.y, __float_as_int(B.z), btab, scr_c32<KIND>(L), scr_nc0<KIND>(L),
                                     finv, nlast);
          dS[0] = fmaf(B.x * w, Lv - B.y, dS[0]);
          T[0] = fmaf(A.z * w, __builtin_amdgcn_logf(Lv * A.w), T[0]);
        }
        p = n_pos;
        for (; p + pstep <= z_end; p += pstep) {
          float4 A = recA[p + hb], B = recB[p + hb];
          int tofs = __float_as_int(B.z);
  #pragma unroll
          for (int t = 0; t < NT; ++t) {
            float Lv = lrf32<KIND, NN>(nd[t], A.x, A.y, tofs, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
            dS[t] = fmaf(B.x, Lv - B.y, dS[t]);
          }
        }
        if (split && p < z_end) {
          float4 A = recA[p], B = recB[p];
          const float w = hb ? 0.f : 1.f;
          float Lv = lrf32<KIND, NN>(nd[0], A.x, A.y, __float_as_int(B.z), btab, scr_c32<KIND>(L), scr_nc0<KIND>(L),
                                     finv, nlast);
          dS[0] = fmaf(B.x * w, Lv - B.y, dS[0]);
        }
        if (split) {
          dS[0] += __shfl_xor(dS[0], 32);
          T[0] += __shfl_xor(T[0], 32);
        }
      }
      // edge sensors (the factored screen has its own loops), whole sums per
      // node lane: a distance within the band
      // of the domain end sends the node to FP64; beyond the end the LRF is
      // zero and the logarithm takes the floor, as in FP64
      bool knife[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) knife[t] = false;
      if constexpr (radial_kind(KIND) && !FA) {
        for (int p = n_ci; p < n_pos; ++p) {
          const float4 A = recA[p], B = recB[p];
          const int o = __float_as_int(B.z);
          const float fw = flf * A.w;
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const float v = rad_v(nd[t], A.x, A.y);
            const float Lv = rad32<NN>(rad_tab<KIND>(nd[t], btab, o), v, nlast);
            knife[t] = knife[t] || fabsf(v - vhi) < band;
            dS[t] = fmaf(B.x, Lv - B.y, dS[t]);
            T[t] = fmaf(A.z, __builtin_amdgcn_logf(fmaxf(Lv * A.w, v >= vhi ? fw : 0.f)), T[t]);
          }
        }
        for (int p = z_end; p < n_scr; ++p) {
          const float4 A = recA[p], B = recB[p];
          const int o = __float_as_int(B.z);
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const float v = rad_v(nd[t], A.x, A.y);
            const float Lv = rad32<NN>(rad_tab<KIND>(nd[t], btab, o), v, nlast);
            knife[t] = knife[t] || fabsf(v - vhi) < band;
            dS[t] = fmaf(B.x, Lv - B.y, dS[t]);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        float S = rel ? Sc + dS[t] : dS[t];
        float lS = rel ? log2_1p(dS[t] * iSc) : __builtin_amdgcn_logf(dS[t]);
        float d = N32 * lS - T[t];
        // a sensor with counts where the screened LRF is 0 (a rounding hole)
        // makes d infinite or NaN: such nodes go to FP64, untrusted, as do
        // nodes at the domain end of an edge sensor
        const bool fin = d < kInf && d > -kInf && !knife[t];
        const bool live = valid[t] && S > 0.f;
        D[t] = (live && fin) ? d : kInf;
        Snode[t] = (live && !fin) ? -1.0f : S;
      }
    } else {
      float S[NT], Q[NT], Ag[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) { S[t] = 0.f; Q[t] = 0.f; }
      if constexpr (FX) {
        // sums, then Pearson terms, over chunks of staged sensors (staged
        // once when every screened sensor fits one chunk)
        const bool one = n_scr <= xcap;
        for (int p0 = 0; p0 < n_scr; p0 += xcap) {
          const int p1 = p0 + xcap < n_scr ? p0 + xcap : n_scr;
          xf_stage(p0, p1 - p0);
          for (int p = p0; p < p1; ++p) {
            const float4 B = recB[p];
            const float* rows = W.xf + (p - p0) * xstride;
#pragma unroll
            for (int t = 0; t < NT; ++t) S[t] = fmaf(B.x, xf_lrf(rows, t), S[t]);
          }
          if (!one) wave_sync_lds();
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) Ag[t] = S[t] > 0.f ? N32 / S[t] : 0.f;
        for (int p0 = 0; p0 < n_scr; p0 += xcap) {
          const int p1 = p0 + xcap < n_scr ? p0 + xcap : n_scr;
          if (!one) xf_stage(p0, p1 - p0);
          for (int p = p0; p < p1; ++p) {
            const float4 A = recA[p], B = recB[p];
            const float* rows = W.xf + (p - p0) * xstride;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              const float mu = Ag[t] * B.x * xf_lrf(rows, t);
              const float dd = A.z - mu;
              const float v = fmaxf(mu, fvf);
              Q[t] = fmaf(dd * dd, __builtin_amdgcn_rcpf(v), Q[t]);
            }
          }
          wave_sync_lds();
        }
      } else {
      int p = 0;
      for (; p + pstep <= n_scr; p += pstep) {
        float4 A = recA[p + hb], B = recB[p + hb];
        int tofs = __float_as_int(B.z);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          float Lv = lrf32<KIND, NN>(nd[t], A.x, A.y, tofs, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
          S[t] = fmaf(B.x, Lv, S[t]);
        }
      }
      if (split && p < n_scr) {
        float4 A = recA[p], B = recB[p];
        float Lv = lrf32<KIND, NN>(nd[0], A.x, A.y, __float_as_int(B.z), btab, scr_c32<KIND>(L), scr_nc0<KIND>(L),
                                   finv, nlast);
        S[0] = fmaf(hb ? 0.f : B.x, Lv, S[0]);
      }
      if (split) S[0] += __shfl_xor(S[0], 32);
#pragma unroll
      for (int t = 0; t < NT; ++t) Ag[t] = S[t] > 0.f ? N32 / S[t] : 0.f;
      for (p = 0; p + pstep <= n_scr; p += pstep) {
        float4 A = recA[p + hb], B = recB[p + hb];
        int tofs = __float_as_int(B.z);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          float Lv = lrf32<KIND, NN>(nd[t], A.x, A.y, tofs, btab, scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
          float mu = Ag[t] * B.x * Lv;
          float dd = A.z - mu;
          float v = fmaxf(mu, fvf);
          Q[t] = fmaf(dd * dd, __builtin_amdgcn_rcpf(v), Q[t]);
        }
      }
      if (split && p < n_scr) {
        float4 A = recA[p], B = recB[p];
        float Lv = lrf32<KIND, NN>(nd[0], A.x, A.y, __float_as_int(B.z), btab, scr_c32<KIND>(L), scr_nc0<KIND>(L),
                                   finv, nlast);
        float mu = Ag[0] * B.x * Lv;
        float dd = A.z - mu;
        float v = fmaxf(mu, fvf);
        Q[0] = fmaf(hb ? 0.f : dd * dd, __builtin_amdgcn_rcpf(v), Q[0]);
      }
      if (split) Q[0] += __shfl_xor(Q[0], 32);
      }
      // nodes at the domain end of an edge sensor go to FP64 (untrusted)
      bool knife[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) knife[t] = false;
      if constexpr (radial_kind(KIND)) {
        auto mark = [&](int p0, int p1) {
          for (int p = p0; p < p1; ++p) {
            const float4 A = recA[p];
#pragma unroll
            for (int t = 0; t < NT; ++t)
              knife[t] = knife[t] || fabsf(rad_v(nd[t], A.x, A.y) - vhi) < band;
          }
        };
        mark(n_ci, n_pos);
        mark(z_end, n_scr);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        Snode[t] = knife[t] ? -1.0f : S[t];
        D[t] = (valid[t] && S[t] > 0.f && Q[t] < kInf && !knife[t]) ? Q[t] : kInf;
      }
    }

    // ---- trusted screen values; best screened node
    // (centre-relative ML values of nodes with S far below S_c suffer
    //  cancellation; such nodes are always re-decided in FP64)
    bool trusted[NT];
    float best = kInf;
    int jb = 1 << 30;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      trusted[t] = (STAT == ANTS_STAT_ML && rel) ? (Snode[t] >= 0.01f * Sc) : !(Snode[t] < 0.f);
      float v = trusted[t] ? D[t] : kInf;
      int j = t * 64 + lane;
      if (v < best || (v == best && j < jb)) { best = v; jb = j; }
    }
    wargmin_f(best, jb);
    best = uni(best);
    jb = uni(jb);

    {
    const ParView Vb = src.view();
    const DevLrf& L = Vb.L;
    const GridP& G = Vb.G;
    const IoP& io = Vb.io;
    // ---- error bound of the screen at the best node (lane-parallel over sensors)
    float margin = 0.f;
    have_prev = best < kInf;
    if (best < kInf) {
      // the best node's screened S and FP32 node description, from its lane
      const int tb = jb >> 6, lb = jb & 63;
      float Sb = 0.f;
      NodeF<KIND> ndb;
      if constexpr (xy_kind(KIND)) {
        double xx, yy, zz;
        make_node<KIND>(L, G, cx, cy, cz, sx, sy, sz, jb, ztab, nodeidx, ndb, xx, yy, zz);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t == tb) {
          Sb = lane_val(Snode[t], lb);
          if constexpr (radial_kind(KIND)) {
            ndb.ox = lane_val(nd[t].ox, lb);
            ndb.oy = lane_val(nd[t].oy, lb);
          }
          if constexpr (KIND == ANTS_LRF_RZ) ndb.tab = ztab + lane_val((int)(nd[t].tab - ztab), lb);
        }
      }
      float Lb[SL];
      float4 RA[SL], RB[SL];
#pragma unroll
      for (int q = 0; q < SL; ++q) {
        int a = lane + 64 * q;
        Lb[q] = 0.f;
        RA[q] = make_float4(0.f, 0.f, 0.f, 1.f);
        RB[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (a < na && !ign[q]) {
          RA[q] = recA[posq[q]];
          RB[q] = recB[posq[q]];
          Lb[q] = lrf32<KIND, NN>(ndb, RA[q].x, RA[q].y, __float_as_int(RB[q].z), btab,
                                  scr_c32<KIND>(L), scr_nc0<KIND>(L), finv, nlast);
        }
        Lprev[q] = Lb[q];
      }
      if (STAT == ANTS_STAT_ML) {
        float A1 = 0.f, A2 = 0.f, A3 = 0.f;
        float iSb = Sb > 0.f ? 1.0f / Sb : 0.f;
#pragma unroll
        for (int q = 0; q < SL; ++q) {
          int a = lane + 64 * q;
          if (a < na && !ign[q]) {
            float mu = N32 * RB[q].x * Lb[q] * iSb;
            A1 += fabsf(mu - RA[q].z);
            A2 += fabsf(RA[q].z * __builtin_amdgcn_logf(fmaxf(Lb[q], flf) * RA[q].w));
            A3 += RB[q].x * fabsf(Lb[q] - RB[q].y);
          }
        }
        A1 = wsum_f(A1);
        A2 = wsum_f(A2);
        A3 = wsum_f(A3);
        float lsr = (rel && Sb > 0.f) ? fabsf(__builtin_amdgcn_logf(Sb * iSc)) : 0.f;
        float E = kU * (kLog2e * (24.f * A1 + 2.f * N32 + (float)(na + 2) * N32 * A3 * iSb) +
                        (float)(na + 4) * A2 + 4.f * N32 * lsr);
        // twice the bound: on 300 k events each of the r-z plain grid and
        // the seeded refinement, decisions first differ from all-FP64 ones
        // at a quarter of the bound
        margin = 2.f * G.margin_scale * E;
      } else {
        float A1 = 0.f;
        float Ab = Sb > 0.f ? N32 / Sb : 0.f;
#pragma unroll
        for (int q = 0; q < SL; ++q) {
          int a = lane + 64 * q;
          if (a < na && !ign[q]) {
            float mu = Ab * RB[q].x * Lb[q];
            float dd = RA[q].z - mu;
            float v = fmaxf(mu, fvf);
            A1 += 2.f * fabsf(dd) + dd * dd / v;
          }
        }
        A1 = wsum_f(A1);
        float E = kU * (float)(24 + na + 4) * A1;
        margin = 4.f * G.margin_scale * E;
      }
      margin = uni(margin);
      if (!(margin < kInf)) margin = kInf;
    }

    // ---- candidates: trusted nodes within the bound, and untrusted valid nodes
    int ncand = 0;
    bool only_trusted = true;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bool c = trusted[t] ? (D[t] < kInf && D[t] <= best + margin)
                          : (valid[t] && Snode[t] > -kInf);
      uint64_t m = __ballot(c);
      if (c) cand[ncand + prefix_count(m)] = (uint16_t)(t * 64 + lane);
      ncand += __popcll(m);
      if (__ballot(c && !trusted[t])) only_trusted = false;
    }
    wave_sync_lds();

    int win = -1;
    bool tie = false;
    if (ncand == 1 && only_trusted) {
      win = jb;
    } else if (ncand > 0) {
      make_rows();
      // one round over the candidates; after a tie, a second round over
      // every valid node (the screen's error bound holds at the best screened
      // node, so a tied node farther out may have screened outside it)
      for (int round = 0; round < 2; ++round) {
        // FP64 values of the candidates: groups of gs lanes per candidate,
        // each lane over every gs-th sensor; gs from a cost model (sensor
        // terms : group reduction steps : per-candidate work = 9 : 1 : 6)
        int gs = 64, best_cost = 1 << 30;
        for (int g = 1; g <= 64; g <<= 1) {
          const int per_pass = 64 / g;
          const int cost = ((ncand + per_pass - 1) / per_pass) *
                           (((na + g - 1) / g) * 9 + (31 - __builtin_clz(g)) + 6);
          if (cost < best_cost) {
            best_cost = cost;
            gs = g;
          }
        }
        const int lgs = uni(31 - __builtin_clz(gs));
        const int sub = lane & ((1 << lgs) - 1);
        const int per_pass = 64 >> lgs;
        double bestd = __builtin_huge_val();
        double* cval = W.cval;
        for (int base = 0; base < ncand; base += per_pass) {
          const int c = base + (lane >> lgs);
          const int j = c < ncand ? (int)cand[c] : (1 << 30);
          double xx = 0.0, yy = 0.0, zz = 0.0;
          bool ok = false;
          const double* zrow = zc64;
          if (c < ncand) {
            NodeF<KIND> ndd;
            ok = make_node<KIND>(L, G, cx, cy, cz, sx, sy, sz, j, ztab, nodeidx, ndd, xx, yy, zz);
            if constexpr (KIND == ANTS_LRF_RZ) zrow = zc64 + (nodeidx[j] >> G.shz) * L.nc0;
          }
          double S = 0.0, T = 0.0;
          if (ok) {
            for (int p = sub; p < na; p += 1 << lgs) {
              const SensorRec64 r = rec64[p];
              const float n = r.n;
              if (n < 0.f) continue;   // ignored by the sensor cuts
              double Lv;
              if constexpr (KIND == ANTS_LRF_RZ) Lv = lrf64_plane(L, r.X, r.Y, xx, yy, zrow);
              else Lv = lrf64s<KIND>(L, r.X, r.Y, r.coff, xx, yy, zz);
              S += r.g * Lv;
              if (STAT == ANTS_STAT_ML && n > 0.f)
                T += (double)n * log(Lv > G.lfloor ? Lv : G.lfloor);
            }
          }
          S = gsum(S, lgs, lane);
          double Dv = __builtin_huge_val();
          if constexpr (STAT == ANTS_STAT_ML) {
            T = gsum(T, lgs, lane);
            if (ok && S > 0.0) Dv = N * log(S) - T;
          } else {
            double Q = 0.0;
            if (ok && S > 0.0) {
              const double Aa = N / S;
              for (int p = sub; p < na; p += 1 << lgs) {
                const SensorRec64 r = rec64[p];
                const float n = r.n;
                if (n < 0.f) continue;   // ignored by the sensor cuts
                double Lv;
                if constexpr (KIND == ANTS_LRF_RZ) Lv = lrf64_plane(L, r.X, r.Y, xx, yy, zrow);
                else Lv = lrf64s<KIND>(L, r.X, r.Y, r.coff, xx, yy, zz);
                const double mu = Aa * r.g * Lv;
                const double dd = (double)n - mu;
                Q += dd * dd / (mu > G.vfloor ? mu : G.vfloor);
              }
            }
            Q = gsum(Q, lgs, lane);
            if (ok && S > 0.0) Dv = Q;
          }
          if (!(Dv < __builtin_huge_val())) Dv = __builtin_huge_val();
          if (sub == 0 && c < ncand) cval[c] = Dv;
          double v1 = Dv;
          int j1 = j;
          wargmin_d(v1, j1);
          bestd = v1 < bestd ? v1 : bestd;
        }
        nfp += ncand;
        wave_sync_lds();
        // values within kTieRel * N of the minimum are equal (their
        // differences are rounding of sums taken in different orders); the
        // lowest node index among them wins.  Candidates are listed in
        // increasing node index, so the first one in the window is the winner.
        if (bestd < __builtin_huge_val()) {
          const double lim = uni(bestd + kTieRel * N);
          int first = -1, nwin = 0;
          for (int c0 = 0; c0 < ncand; c0 += 64) {
            const int c = c0 + lane;
            const uint64_t m = __ballot(c < ncand && cval[c] <= lim);
            if (first < 0 && m) first = c0 + __builtin_ctzll(m);
            nwin += __popcll(m);
          }
          win = uni((int)cand[uni(first)]);
          tie = nwin > 1;
        }
        if (round == 0 && tie) {
          int nall = 0;
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            const uint64_t m = __ballot(valid[t]);
            if (valid[t]) cand[nall + prefix_count(m)] = (uint16_t)(t * 64 + lane);
            nall += __popcll(m);
          }
          wave_sync_lds();
          if (nall > ncand) {
            ncand = nall;
            continue;
          }
        }
        break;
      }
    }
    if (io.path && lane == 0 && k < G.K) io.path[e * G.K + k] = win;
    if (win < 0) {
      status |= ANTS_EV_NO_VALID_NODE;
    } else {
      if (tie) status |= ANTS_EV_TIE;
      const int pk = uni((int)nodeidx[win]);
      const int jx = pk & G.mskx, jy = (pk >> G.shy) & G.msky, jz = pk >> G.shz;
      cx = uni(cx + (double)(jx - G.hx) * sx);
      cy = uni(cy + (double)(jy - G.hy) * sy);
      cz = uni(cz + (double)(jz - G.hz) * sz);
    }
    sx = uni(sx * G.shrink);
    sy = uni(sy * G.shrink);
    sz = uni(sz * G.shrink);
    wave_sync_lds();
    }
  }

  // ---------------- outputs at the final centre, FP64, lane-parallel over sensors
  const ParView Vo = src.view();
  {
  const DevLrf& L = Vo.L;
  const GridP& G = Vo.G;
  const IoP& io = Vo.io;
  double S = 0.0;
  double Lf[SL];
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    int a = lane + 64 * q;
    Lf[q] = 0.0;
    if (a < na && !ign[q]) {
      Lf[q] = lrf64<KIND>(L, a, cx, cy, cz);
      S += L.g[a] * Lf[q];
    }
  }
  S = wsum_d(S);
  double Aa = N / S, ll = 0.0, q2 = 0.0;
  bool okS = S > 0.0 && S < __builtin_huge_val();
  if (okS) {
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      int a = lane + 64 * q;
      if (a < na && !ign[q]) {
        double mu = Aa * L.g[a] * Lf[q];
        double Lt = Lf[q] > G.lfloor ? Lf[q] : G.lfloor;
        double n = (double)nq[q];
        if (n > 0.0) ll += n * log(Aa * L.g[a] * Lt);
        ll -= mu;
        double dd = n - mu;
        q2 += dd * dd / (mu > G.vfloor ? mu : G.vfloor);
      }
    }
    ll = wsum_d(ll);
    q2 = wsum_d(q2);
  }
  if (io.path && Kev < G.K && lane >= Kev && lane < G.K) io.path[e * G.K + lane] = -1;
  status |= G.or_status;
  if (lane == 0) {
    if (G.fb_thr >= 0.0 && !(okS && ndf > 0 && q2 / ndf <= G.fb_thr)) {
      int slot = atomicAdd(io.fb_count, 1);
      io.fb_list[slot] = (int32_t)e;
    }
    float nan = __builtin_nanf("");
    io.x[e] = (float)cx;
    io.y[e] = (float)cy;
    io.z[e] = (float)cz;
    io.E[e] = okS ? (float)Aa : nan;
    io.lnl[e] = okS ? (float)ll : nan;
    io.chi2[e] = okS ? (float)q2 : nan;
    io.ndf[e] = ndf;
    io.status[e] = status;
    if (io.nfp) io.nfp[e] = nfp;
  }
  }
}

// Occupancy target: four waves per SIMD (128 VGPRs) for one node tile,
// whose time goes largely to latency-bound reductions and FP64 decisions;
// three (168 VGPRs) for more tiles; the XY kernels with many tiles keep two.
template <int KIND, int NT>
constexpr int waves_per_eu() { return (xy_kind(KIND) && NT >= 4) ? 2 : NT == 1 ? 4 : 3; }

template <int KIND, int STAT, int NT, int SL, bool NN, int FZ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves_per_eu<KIND, NT>())))
cg_kernel(KArgs A) {
  KArgsK* kp0 = (KArgsK*)__builtin_amdgcn_kernarg_segment_ptr();
  const DevLrf& L = A.L;
  const GridP& G = A.G;
  const IoP& io = A.io;
  const int64_t waves_total = A.waves_total;
  const int per_wave_bytes = A.per_wave_bytes, btab_n = A.btab_n;
  extern __shared__ float4 smem4[];
  // block-shared table: axial pp tables, or r-z r-polynomials per z-row
  float4* btab = smem4;
  for (int i = threadIdx.x; i < btab_n; i += blockDim.x) btab[i] = ((const float4*)L.pp)[i];
  __syncthreads();
  const int lane0 = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nwb = blockDim.x >> 6;
  unsigned char* wbase = (unsigned char*)(smem4 + btab_n) + (size_t)wv * per_wave_bytes;
  wave_setup<KIND, NT, (FZ > 0 && KIND == ANTS_LRF_RZ), (FZ > 0 && KIND == ANTS_LRF_XY)>(
      wbase, L, G, lane0);
  int64_t nwork = io.list ? (int64_t)(*io.list_n) : io.n;
  // one node tile (small grids, the seeded refinement): parameters re-read
  // per event and stage (measured 3.5% faster); more tiles: held in
  // registers (measured 4% faster than re-reading)
  auto event = [&](int64_t e) {
    if constexpr (NT == 1)
      process_event<KIND, STAT, NT, SL, NN, FZ>(KargSrc{kp0}, e, btab, wbase, opaque(lane0));
    else
      process_event<KIND, STAT, NT, SL, NN, FZ>(RefSrc{L, G, io}, e, btab, wbase, opaque(lane0));
  };
  if ((gridDim.x & 7) == 0) {
    // workgroups go round-robin to the 8 XCDs, each with its own L2: block b
    // runs on XCD b % 8.  Each XCD takes whole runs of 32 consecutive work
    // items (a 128-byte line of every 4-byte output array, and neighbouring
    // signal rows), its waves striding over them, so lines are not split
    // between L2s.
    const int64_t x = blockIdx.x & 7;
    const int64_t nwx = (int64_t)(gridDim.x >> 3) * nwb;
    for (int64_t i = (int64_t)(blockIdx.x >> 3) * nwb + wv;; i += nwx) {
      const int64_t w = (((i >> 5) << 3) + x) * 32 + (i & 31);
      if (w >= nwork) break;
      const int64_t e = io.list ? (int64_t)io.list[w] : w;
      event(e);
    }
  } else {
    for (int64_t w = (int64_t)blockIdx.x * nwb + wv; w < nwork; w += waves_total) {
      const int64_t e = io.list ? (int64_t)io.list[w] : w;
      event(e);
    }
  }
}

template <int KIND, int STAT, int NT, int SL, bool NN, int FZ = 0>
hipError_t launch_t(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t stream,
                    int max_blocks) {
  int btab_n = 0;
  if (KIND == ANTS_LRF_AXIAL || KIND == ANTS_LRF_COMPOSITE) btab_n = L.ntab * L.nintp;
  if (KIND == ANTS_LRF_RZ) btab_n = L.nc1 * L.nintp;
  constexpr bool fa = FZ > 0 && KIND == ANTS_LRF_RZ, fx = FZ > 0 && KIND == ANTS_LRF_XY;
  const int per_wave = wave_lds_bytes(KIND, L.na, G.nz, L.nintp, L.nc0, NT, fa ? G.nx * G.ny : 0) +
                       (fx ? kXfBytes : 0);
  // waves (events in flight) per block and a cap on resident blocks per
  // CU from the set's launch plan
  const int wpb = (G.plan_wpb >= 1 && G.plan_wpb <= kWavesPerBlock) ? G.plan_wpb : kWavesPerBlock;
  if (G.plan_bpc > 0 && (int64_t)G.plan_bpc * num_cu() < max_blocks)
    max_blocks = G.plan_bpc * num_cu();
  size_t smem = (size_t)btab_n * 16 + (size_t)wpb * per_wave;
  int64_t nwork = io.n;
  int64_t blocks = (nwork + wpb - 1) / wpb;
  auto kern = cg_kernel<KIND, STAT, NT, SL, NN, FZ>;
  if (smem > 65536) {
    hipError_t st = hipFuncSetAttribute((const void*)kern,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (st != hipSuccess) return st;
  }
  // waves stride over the events: launch no more blocks than are resident
  // at once, so that no block starts after the others have finished
  int resident = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, kern, 64 * wpb, smem) ==
          hipSuccess &&
      resident > 0 && (int64_t)resident * num_cu() < max_blocks)
    max_blocks = resident * num_cu();
  if (blocks > max_blocks) blocks = max_blocks;
  if (blocks < 1) blocks = 1;
  if (blocks > 8) blocks = blocks / 8 * 8;   // XCD-aware work order (see cg_kernel)
  int64_t waves_total = blocks * wpb;
  KArgs A{L, G, io, waves_total, per_wave, btab_n};
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * wpb), smem, stream, A);
  return hipGetLastError();
}

// factored screens: r-z column-factored for FZ z-planes; XY (FZ = 1) from
// y-collapsed rows staged in LDS
template <int KIND, int STAT, int SL, bool NN, int FZ>
hipError_t launch_fz(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t s, int mb) {
  switch (node_tiles(G.nn)) {
    case 1: return launch_t<KIND, STAT, 1, SL, NN, FZ>(L, G, io, s, mb);
    case 2: return launch_t<KIND, STAT, 2, SL, NN, FZ>(L, G, io, s, mb);
    case 4: return launch_t<KIND, STAT, 4, SL, NN, FZ>(L, G, io, s, mb);
    case 6: return launch_t<KIND, STAT, 6, SL, NN, FZ>(L, G, io, s, mb);
    default: return launch_t<KIND, STAT, 8, SL, NN, FZ>(L, G, io, s, mb);
  }
}

template <int KIND, int STAT, int SL, bool NN>
hipError_t launch_kss(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t s, int mb) {
  // r-z, ML: the column-factored screen for 3, 5 or 7 z planes, unless
  // the launch plan asks for the per-node screen
  if constexpr (KIND == ANTS_LRF_RZ && STAT == ANTS_STAT_ML && SL == 1) {
    if (G.plan_screen != 1) {
      if (G.nz == 3) return launch_fz<KIND, STAT, SL, NN, 3>(L, G, io, s, mb);
      if (G.nz == 5) return launch_fz<KIND, STAT, SL, NN, 5>(L, G, io, s, mb);
      if (G.nz == 7) return launch_fz<KIND, STAT, SL, NN, 7>(L, G, io, s, mb);
    }
  }
  if constexpr (KIND == ANTS_LRF_XY) {
    if (G.plan_screen != 1 && xf_applies(L, G)) return launch_fz<KIND, STAT, SL, NN, 1>(L, G, io, s, mb);
  }
  switch (node_tiles(G.nn)) {
    case 1: return launch_t<KIND, STAT, 1, SL, NN>(L, G, io, s, mb);
    case 2: return launch_t<KIND, STAT, 2, SL, NN>(L, G, io, s, mb);
    case 4: return launch_t<KIND, STAT, 4, SL, NN>(L, G, io, s, mb);
    case 6: return launch_t<KIND, STAT, 6, SL, NN>(L, G, io, s, mb);
    default: return launch_t<KIND, STAT, 8, SL, NN>(L, G, io, s, mb);
  }
}

template <int KIND, int STAT, bool NN>
hipError_t launch_ksn(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t s, int mb) {
  if (L.na <= 64) return launch_kss<KIND, STAT, 1, NN>(L, G, io, s, mb);
  if (L.na <= 128) return launch_kss<KIND, STAT, 2, NN>(L, G, io, s, mb);
  return launch_kss<KIND, STAT, 4, NN>(L, G, io, s, mb);
}

template <int KIND, int STAT>
hipError_t launch_ks(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t s, int mb) {
  if constexpr (radial_kind(KIND)) {
    if (L.nonneg) return launch_ksn<KIND, STAT, true>(L, G, io, s, mb);
  }
  return launch_ksn<KIND, STAT, false>(L, G, io, s, mb);
}


// ------------------------------------------------- persistent multi-detector

// One launch over event chunks from several detectors (LRF sets): waves pull
// work items (chunk, tile of its set's T events) from device counters until
// the stream is exhausted; every wave leaves the loop once the counters pass
// the last item.  Per set: events per item, tables in LDS or through the
// cache, and the fewest sensor slots per lane that hold its sensors (the
// kernel carries the event code for each slot count up to SL).
template <int KIND, int STAT, int NT, int SL, bool NN>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(waves_per_eu<KIND, NT>()))) cg_multi_kernel(MultiP P) {
  extern __shared__ float4 smem4[];
  float4* btab = smem4;
  for (int si = 0; si < P.n_sets; ++si) {
    const int off = P.sets[si].tab_off;
    if (off < 0) continue;
    const DevLrf& L = P.sets[si].L;
    const int n = KIND == ANTS_LRF_AXIAL ? L.ntab * L.nintp : KIND == ANTS_LRF_RZ ? L.nc1 * L.nintp : 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) btab[off + i] = ((const float4*)L.pp)[i];
  }
  __syncthreads();
  const int lane0 = lane_id();
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned char* wbase = (unsigned char*)(smem4 + P.btab_n) + (size_t)wv * P.per_wave_bytes;
  int cur_set = -1;
  // XCD-aware claims (the grid is a multiple of 8 blocks; block b runs on
  // XCD b % 8, each with its own L2): runs of G items covering 32 output
  // rows belong to one XCD, claimed through that XCD's counter; a wave whose
  // XCD has none left takes the other XCDs' items in turn
  const int G = P.xg;
  const int x0 = blockIdx.x & 7;
  int xs = 0;
  for (;;) {
    int item = -1;
    while (xs < 8) {
      const int x = (x0 + xs) & 7;
      int k = 0;
      if (lane0 == 0) k = atomicAdd(P.counter + 16 * x, 1);
      k = lane_val(k, 0);
      const int64_t i = ((int64_t)(k / G) * 8 + x) * G + (k % G);
      if (i < P.n_items) {
        item = (int)i;
        break;
      }
      ++xs;
    }
    if (item < 0) break;
    int lo = 0, hi = P.n_chunks;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (P.prefix[mid] <= item) lo = mid;
      else hi = mid;
    }
    lo = uni(lo);
    const ChunkDesc ch = P.chunks[lo];
    const SetDesc& sd = P.sets[ch.set];
    if (ch.set != cur_set) {
      cur_set = ch.set;
      wave_setup<KIND, NT>(wbase, sd.L, sd.G, lane0);
    }
    IoP io = P.out;
    io.sig = ch.sig;
    io.ld = sd.L.ns;
    io.n = ch.n;
    io.x += ch.out_off;
    io.y += ch.out_off;
    io.z += ch.out_off;
    io.E += ch.out_off;
    io.lnl += ch.out_off;
    io.chi2 += ch.out_off;
    io.ndf += ch.out_off;
    io.status += ch.out_off;
    const int toff = uni(sd.tab_off), T = uni(sd.T);
    const float4* tb = toff >= 0 ? btab + toff : (const float4*)sd.L.pp;
    const int64_t e0 = (int64_t)(item - P.prefix[lo]) * T;
    const int64_t e1 = e0 + T < ch.n ? e0 + T : ch.n;
    // sensor slots per lane for this set: the fewest that hold its sensors
    const int na = uni(sd.L.na);
    for (int64_t e = e0; e < e1; ++e) {
      if (SL >= 2 && na <= 64)
        process_event<KIND, STAT, NT, 1, NN, 0>(RefSrc{sd.L, sd.G, io}, e, tb, wbase,
                                                opaque(lane0));
      else if (SL >= 4 && na <= 128)
        process_event<KIND, STAT, NT, (SL >= 4 ? 2 : SL), NN, 0>(RefSrc{sd.L, sd.G, io}, e, tb,
                                                                wbase, opaque(lane0));
      else
        process_event<KIND, STAT, NT, SL, NN, 0>(RefSrc{sd.L, sd.G, io}, e, tb, wbase,
                                                 opaque(lane0));
    }
  }
}

template <int KIND, int STAT, int NT, int SL, bool NN>
hipError_t launch_multi_t(const MultiP& P, int blocks, hipStream_t stream) {
  size_t smem = (size_t)P.btab_n * 16 + (size_t)kWavesPerBlock * P.per_wave_bytes;
  auto kern = cg_multi_kernel<KIND, STAT, NT, SL, NN>;
  if (smem > 65536) {
    hipError_t st = hipFuncSetAttribute((const void*)kern,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
    if (st != hipSuccess) return st;
  }
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(64 * kWavesPerBlock), smem, stream, P);
  return hipGetLastError();
}

template <int KIND, int STAT, int SL, bool NN>
hipError_t launch_multi_ks(const MultiP& P, int nn, int blocks, hipStream_t s) {
  switch (node_tiles(nn)) {
    case 1: return launch_multi_t<KIND, STAT, 1, SL, NN>(P, blocks, s);
    case 2: return launch_multi_t<KIND, STAT, 2, SL, NN>(P, blocks, s);
    case 4: return launch_multi_t<KIND, STAT, 4, SL, NN>(P, blocks, s);
    case 6: return launch_multi_t<KIND, STAT, 6, SL, NN>(P, blocks, s);
    default: return launch_multi_t<KIND, STAT, 8, SL, NN>(P, blocks, s);
  }
}

template <int KIND, int STAT, bool NN>
hipError_t launch_multi_kn(const MultiP& P, int nn, int na, int blocks, hipStream_t s) {
  if (na <= 64) return launch_multi_ks<KIND, STAT, 1, NN>(P, nn, blocks, s);
  if (na <= 128) return launch_multi_ks<KIND, STAT, 2, NN>(P, nn, blocks, s);
  return launch_multi_ks<KIND, STAT, 4, NN>(P, nn, blocks, s);
}

template <int KIND>
hipError_t launch_multi_k(const MultiP& P, int stat, int nn, int na, bool nonneg, int blocks,
                          hipStream_t s) {
  const bool nnz = KIND != ANTS_LRF_XY && nonneg;
  if (stat == ANTS_STAT_ML)
    return nnz ? launch_multi_kn<KIND, 0, true>(P, nn, na, blocks, s)
               : launch_multi_kn<KIND, 0, false>(P, nn, na, blocks, s);
  return nnz ? launch_multi_kn<KIND, 1, true>(P, nn, na, blocks, s)
             : launch_multi_kn<KIND, 1, false>(P, nn, na, blocks, s);
}

// launcher of one LRF kind: ML or chi2 statistic, node tiles, sensor slots,
// non-negative tables
template <int KIND>
hipError_t launch_grid_k(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t s, int mb) {
  return G.stat == ANTS_STAT_ML ? launch_ks<KIND, 0>(L, G, io, s, mb)
                                : launch_ks<KIND, 1>(L, G, io, s, mb);
}

}  // namespace
}  // namespace ants
