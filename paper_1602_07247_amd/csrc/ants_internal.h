// Internal declarations shared by the host API and the HIP kernels of the
// contracting-grid reconstruction library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ants.h"

namespace ants {

constexpr int kMaxSensors = 256;     // row length limit (4 sensor slots per lane)
constexpr int kSlots = kMaxSensors / 64;
constexpr int kMaxNodes = 512;       // 8 tiles of 64 nodes
constexpr int kWavesPerBlock = 4;

// Device-resident view of an LRF set.  Sensors are the active ones only,
// in their original order ("compact index" a = 0..na-1).
struct DevLrf {
  int kind;            // ANTS_LRF_*
  int shared;
  int ns, na;          // row length, active count
  int nb0, nb1;        // breakpoints per axis (nb1 = 1 for axial)
  int nc0, nc1;        // coefficients per axis (nc1 = 1 for axial)
  int nintp;           // FP32 piecewise-polynomial intervals per r-row, incl.
                       // one all-zero interval past the end of the domain
  int ntab;            // number of coefficient tables
  double lo0, hi0, lo1, hi1;
  double d0, d1;       // breakpoint spacing
  float finv0;         // 1/d0 (axial and r-z: lo0 = 0)
  const int32_t* col;  // [na] column of the active sensor in a signal row
  const int32_t* tab;  // [na] coefficient table of the sensor
  const double* X;     // [na] sensor centre
  const double* Y;     // [na]
  const double* g;     // [na] relative gain
  const float* pp;     // axial: [ntab][nintp][4]; r-z: [nc1][nintp][4] (r-polys per z-row)
  const float* c32;    // XY: [ntab][nc1][nc0] FP32 B-spline coefficients
  const double* c64;   // all kinds: [ntab][nc1][nc0] FP64 coefficients
};

struct GridP {
  int nx, ny, nz, nn;  // nodes per axis, total
  int hx, hy, hz;      // (n-1)/2
  int K;               // iterations
  int dim;             // 2 or 3
  int stat;            // ANTS_STAT_*
  int start;           // ANTS_START_*
  double shrink;
  double s0x, s0y, s0z;
  double z_start;
  double lfloor, vfloor;
  float margin_scale;  // multiplier on the screening error bound
};

struct IoP {
  const float* sig;    // [n][ns]
  int64_t ld;          // row stride (elements)
  const float* seeds;  // [n][4] or NULL
  float *x, *y, *z, *E, *lnl, *chi2;
  int32_t *ndf, *status, *path, *nfp;
  int64_t n;           // events (work items when list == NULL)
  const int32_t* list;     // optional: event indices to process
  const int32_t* list_n;   // optional: device count of list entries
};

struct GenP {
  int64_t n;           // events
  uint64_t first;      // global index of the first event (Philox counter)
  uint32_t k0, k1;     // Philox key (seed)
  int region;          // 0 disc, 1 square
  int noiseless;
  double extent, z_lo, z_hi, e_lo, e_hi;
  float* sig;          // [n][ns]
  float* truth;        // [n][4] or NULL
};

hipError_t launch_gen(const DevLrf& L, const GenP& P, hipStream_t stream, int max_blocks);

// Launch the contracting-grid kernel; returns a hipError_t.
hipError_t launch_grid(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t stream,
                       int max_blocks);

}  // namespace ants
