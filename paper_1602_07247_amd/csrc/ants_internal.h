// Internal declarations shared by the host API and the HIP kernels of the
// contracting-grid reconstruction library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "ants.h"

namespace ants {

// status bits of a failed event (EMPTY | BAD_INPUT | NO_ACTIVE | NO_VALID_NODE);
// TIE and FALLBACK describe how a valid position was found
constexpr int kEvFailed = ANTS_EV_EMPTY | ANTS_EV_BAD_INPUT | ANTS_EV_NO_ACTIVE |
                          ANTS_EV_NO_VALID_NODE;
constexpr int kMaxSensors = 256;     // row length limit (4 sensor slots per lane)
constexpr int kSlots = kMaxSensors / 64;
constexpr int kMaxNodes = 512;       // 8 tiles of 64 nodes
constexpr int kWavesPerBlock = 4;
constexpr int kMaxSeedSteps = 16;   // iteration counts a seed's spread may select

// Tiles of 64 node lanes used for a grid of nn nodes (the event kernels
// are instantiated for these counts).
__host__ __device__ constexpr int node_tiles(int nn) {
  return nn <= 64 ? 1 : nn <= 128 ? 2 : nn <= 256 ? 4 : nn <= 384 ? 6 : 8;
}

// Per-wave LDS bytes of the event kernels: sensor records (32 B per active
// sensor, rewritten every iteration, and 32 B of FP64 data per event); for
// r-z the FP32 plane tables (16 B per plane and interval),
// which the FP64 spline rows (8 B per plane and r-coefficient) overlay
// during the FP64 decisions, and the plane weights (16 B FP32 + 32 B FP64
// + 4 B first z-coefficient per plane); 16-bit candidate list and
// node-index table of 64 entries per node tile; the per-axis steps for
// each iteration count a seed may select; for the column-factored r-z
// screen (fact_nxy = nodes per z-plane, 0 = not used) the partial sums of
// every (column, sensor group) and a lane -> (column, group) table.
// Where a wave keeps the FP64 values of its decision candidates (8 bytes
// for each of up to 64 * nt nodes): over the FP32 sensor records (32 bytes
// per sensor) or over the factored screen's partial sums, both dead while
// the candidates are decided; otherwise in a region of its own.
// 0 = own region, 1 = sensor records, 2 = factored-screen sums.
__host__ __device__ inline int cval_place(int na, int nz, int nt, int fact_nxy) {
  const int need = 512 * nt;
  if (32 * na >= need) return 1;
  if (fact_nxy > 0 && 8 * nz * (fact_nxy > 64 ? fact_nxy : 64) >= need) return 2;
  return 0;
}
__host__ __device__ inline int wave_lds_bytes(int kind, int na, int nz, int nintp, int nc0, int nt,
                                              int fact_nxy = 0) {
  int b = 64 * na + 256 * nt + 24 * kMaxSeedSteps;
  if (cval_place(na, nz, nt, fact_nxy) == 0) b += 512 * nt;
  if (fact_nxy > 0) b += 8 * nz * (fact_nxy > 64 ? fact_nxy : 64) + 128;
  if (kind == ANTS_LRF_RZ) {
    const int zt = 16 * nz * nintp, zr = 8 * nz * nc0;
    b += ((zt > zr ? zt : zr) + 15) / 16 * 16 + 52 * nz;
  }
  return (b + 15) & ~15;
}

// XY factored screen: per wave, the y-collapsed coefficient rows of a chunk
// of sensors (kXfFloats floats), and the y-weights and first coefficient
// row of up to 64 node rows.
constexpr int kXfFloats = 1536;
constexpr int kXfBytes = 4 * kXfFloats + 64 * 16 + 64 * 4;

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
  double inv_d0;       // 1/d0 in FP64 (screen distances are kept in units of d0)
  double inv_d1;       // 1/d1 in FP64
  int nonneg;          // every FP32 cubic piece is >= 0 on [0, 1] (no clamp needed)
  const int32_t* col;  // [na] column of the active sensor in a signal row
  const int32_t* tab;  // [na] coefficient table of the sensor
  const double* X;     // [na] sensor centre
  const double* Y;     // [na]
  const double* g;     // [na] relative gain
  const float* pp;     // axial: [ntab][nintp][4]; r-z: [nc1][nintp][4] (r-polys per z-row)
  const float* c32;    // XY: [ntab][nc1][nc0] FP32 B-spline coefficients;
                       // sliced: [ntab][nplanes][nc1][nc0]
  const double* c64;   // all kinds: [ntab][nc1][nc0] FP64 coefficients (sliced:
                       // [ntab][nplanes][nc1][nc0]; composite: the axial row)
  // composite: the XY residual (coefficient tables in xc32 / xc64, table of
  // active sensor a at xtab[a] * xnc0 * xnc1)
  int xnb0, xnb1, xnc0, xnc1;
  double xlo0, xhi0, xlo1, xhi1, xinv_d0, xinv_d1;
  const int32_t* xtab;
  const float* xc32;
  const double* xc64;
  // sliced: planes at zlo + p / inv_dz, p = 0 .. nplanes - 1
  int nplanes;
  double zlo, zhi, inv_dz;
};
// LRF kinds whose screen value is a cubic in the distance r read from a
// table (the domain-end handling of the screen applies to them)
__host__ __device__ constexpr bool radial_kind(int k) {
  return k == ANTS_LRF_AXIAL || k == ANTS_LRF_RZ;
}
// LRF kinds with a bicubic in global x, y (per-node cell and weights)
__host__ __device__ constexpr bool xy_kind(int k) {
  return k == ANTS_LRF_XY || k == ANTS_LRF_COMPOSITE || k == ANTS_LRF_SLICED;
}

struct GridP {
  int nx, ny, nz, nn;  // nodes per axis, total
  int hx, hy, hz;      // (n-1)/2
  int shy, shz;        // node index packing: jx | jy << shy | jz << shz
  int mskx, msky;      // (1 << bits of nx) - 1, (1 << bits of ny) - 1
  int K;               // iterations
  int dim;             // 2 or 3
  int stat;            // ANTS_STAT_*
  int start;           // ANTS_START_*
  double shrink;
  double s0x, s0y, s0z;
  double z_start;
  double lfloor, vfloor;
  float margin_scale;  // multiplier on the screening error bound
  // per-event steps from a seed's log-variance (refinement of a learned seed)
  int seed_steps;
  double kappa;        // initial step >= kappa * predicted sigma
  int kmin, kmax;      // iteration count range
  double sscale[3];    // mm per unit of the seed's standard deviation, per axis
  double sfinal[3];    // final step per axis (= step0 * shrink^(iterations-1))
  double cut_signal;   // > 0: ignore sensors with a signal below it
  double cut_dist;     // > 0: ignore sensors farther (x-y) than it from the start
  double fb_thr;       // >= 0: events with chi2/ndf above it go to the fallback list
  int or_status;       // status bits OR-ed into every processed event
  // launch plan (host side; see ants_grid_plan): waves per block (0 = 4),
  // cap on blocks per CU (0 = as many as fit), screen (0 = factored where it
  // applies: r-z columns, or XY rows staged in LDS; 1 = per node)
  int plan_wpb, plan_bpc, plan_screen;
};

// The XY factored screen applies to single-plane grids of at most 64 node
// columns and rows whose y-collapsed rows of one sensor fit the staging area
// (at most nc0 coefficients per row).
inline bool xf_applies(const DevLrf& L, const GridP& G) {
  return L.kind == ANTS_LRF_XY && G.nz == 1 && G.nx <= 64 && G.ny <= 64 &&
         G.ny * L.nc0 <= kXfFloats;
}

struct IoP {
  const float* sig;    // [n][ns]
  int64_t ld;          // row stride (elements)
  const float* seeds;  // [n][4] or NULL
  float *x, *y, *z, *E, *lnl, *chi2;
  int32_t *ndf, *status, *path, *nfp;
  int64_t n;           // events (work items when list == NULL)
  const int32_t* list;     // optional: event indices to process
  const int32_t* list_n;   // optional: device count of list entries
  int32_t* fb_list;        // fallback list (when G.fb_thr >= 0)
  int32_t* fb_count;       // its device counter
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

// ------------------------------------------------- persistent multi-detector
struct SetDesc {
  DevLrf L;
  GridP G;
  int tab_off;         // float4 offset of the set's table in the block's LDS, or -1:
                       // the table is read through the cache
  int T;               // events per work item of this set's chunks
};
struct ChunkDesc {
  const float* sig;    // [n][ns of its set]
  int64_t n;
  int64_t out_off;     // first output row
  int32_t set;
  int32_t pad_;
};
struct MultiP {
  const SetDesc* sets;
  int n_sets;
  const ChunkDesc* chunks;
  const int32_t* prefix;   // [n_chunks + 1] first work item of each chunk
  int n_chunks;
  int n_items;
  int xg;                  // work items per run claimed on one XCD
  int* counter;            // 8 work counters, 16 ints apart (zeroed before the launch)
  IoP out;                 // output arrays (offset per chunk)
  int per_wave_bytes;
  int btab_n;              // float4 entries of the sets' tables staged in LDS
};
hipError_t launch_multi(const MultiP& P, int kind, int stat, int max_nn, int max_na, bool nonneg,
                        int blocks, hipStream_t s);

// ------------------------------------------------------------ learned seed
struct GemmP {
  int M, N, K;
  const __bf16* A;
  int64_t sa_m, sa_k;  // A(m, k) = A[m * sa_m + k * sa_k]
  const __bf16* B;
  int64_t sb_n, sb_k;  // B(n, k)
  const float* bias;   // [N] or NULL
  int relu;
  const __bf16* mask;  // zero C where mask(m, n) <= 0 (ReLU derivative) or NULL
  int64_t ldmask;
  float* Cf;           // FP32 result or NULL
  int64_t ldcf;
  __bf16* Cb;          // BF16 result or NULL
  int64_t ldcb;
  // optional FP32 workspace for split-K partial products (ws_n floats);
  // NULL: no split
  float* ws;
  int64_t ws_n;
};
// Split of the k range for a GEMM whose output has few 64 x 64 tiles and a
// long k (weight gradients, k = batch): enough splits to give about 256
// blocks, each at least 64 deep.
inline int gemm_splits(int M, int N, int K) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  if (tiles >= 128 || K < 128) return 1;
  int s = (256 + tiles - 1) / tiles;
  if (s > K / 64) s = K / 64;
  if (s > 64) s = 64;
  return s < 1 ? 1 : s;
}
struct HeadP {
  float scale[3], inv_scale[3], offset[3];
  float inv_batch;
};
struct AdamP {
  float lr, b1, b2, eps, c1, c2;   // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
};
hipError_t launch_gemm(const GemmP& P, hipStream_t s);
hipError_t launch_normalize(const float* sig, int64_t ld, const int32_t* col, int na, int64_t n,
                            int kin, __bf16* X, hipStream_t s);
hipError_t launch_head_loss(const float* Y, const float* target, int64_t ldt, int64_t n,
                            const HeadP& H, float* dY, __bf16* dYb, float* loss, hipStream_t s);
hipError_t launch_head_back(const float* dY, const float* W4, const __bf16* H3, int64_t n,
                            int hidden, __bf16* dH, hipStream_t s);
hipError_t launch_colsum_bf16(const __bf16* D, int64_t n, int ld, int cols, float* out,
                              hipStream_t s);
hipError_t launch_colsum_f32(const float* D, int64_t n, int ld, int cols, float* out,
                             hipStream_t s);
hipError_t launch_sum_f32(const float* v, int64_t n, float scale, float* out, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, __bf16* pb, int64_t n,
                       const AdamP& A, hipStream_t s);
hipError_t launch_to_bf16(const float* p, __bf16* pb, int64_t n, hipStream_t s);
// Fused inference (hidden width 256): normalisation, every layer and the
// output layer in one kernel; out = raw outputs (seeds = 0) or seeds in mm
// with the log-variance (seeds = 1).
constexpr int kFwdMaxLayers = 4;
struct FwdP {
  const float* sig;
  int64_t ld;
  const int32_t* col;
  int na;
  int64_t n;
  int kin;                              // padded input width (multiple of 32, <= 256)
  int layers;                           // hidden layers
  const __bf16* W[kFwdMaxLayers + 1];   // BF16 weights [out][in], output layer last
  const float* b[kFwdMaxLayers + 1];    // FP32 biases
  float* out;                           // [n][4]
  int seeds;
  float scale[3], offset[3];
};
hipError_t launch_mlp_fwd(const FwdP& P, hipStream_t s);

// Launch the contracting-grid kernel; returns a hipError_t.
hipError_t launch_grid(const DevLrf& L, const GridP& G, const IoP& io, hipStream_t stream,
                       int max_blocks);

// ------------------------------------------------------------ host side
// error reporting (message kept for ants_last_error)
ants_status set_error(ants_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ants_status hip_error(hipError_t e, const char* what);
// ants_grid_cfg -> kernel parameters (validated against the LRF set)
ants_status grid_params(const DevLrf& L, const ants_grid_cfg* cfg, GridP* G);
// key of a grid configuration in a set's plan cache (fields that change the
// work per event); never 0
uint64_t grid_cfg_key(const ants_grid_cfg& c);
// the set's stored launch plan for this configuration, if any, into G
void apply_grid_plan(const ants_lrfset* S, const ants_grid_cfg* cfg, GridP* G);
int num_cu();
// grow-only device buffer
hipError_t ensure(void** p, size_t* have, size_t need);
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int64_t n, hipStream_t s);

}  // namespace ants

struct ants_lrfset {
  ants::DevLrf d;
  int device;
  int ns;
  std::vector<void*> allocs;
  // host copy of the descriptor (ants_lrfset_save)
  int32_t h_kind = 0, h_shared = 0, h_knots[2] = {0, 0};
  double h_lo[2] = {0, 0}, h_hi[2] = {0, 0};
  std::vector<double> h_xy, h_gain, h_coef;
  std::vector<uint8_t> h_active;
  // workspace of the seeded reconstruction (seeds, fallback list, counter)
  void* ws_seeds = nullptr;
  size_t ws_seeds_bytes = 0;
  void* ws_list = nullptr;
  size_t ws_list_bytes = 0;
  int32_t* ws_count = nullptr;
  // workspace of the multi-detector launch (descriptors, counter), its
  // pinned host staging and the event that marks the end of the last copy
  // from it
  void* ws_multi = nullptr;
  size_t ws_multi_bytes = 0;
  void* ms_host = nullptr;
  size_t ms_host_bytes = 0;
  hipEvent_t ms_copied = nullptr;
  // launch plans of ants_reconstruct per grid configuration (ants_autotune,
  // ants_set_plan): key, waves per block, blocks per CU, screen
  struct GridPlanEntry {
    uint64_t key;
    int32_t wpb, bpc, screen;
  };
  GridPlanEntry gplan[8] = {};
  int n_gplan = 0;
  // this set's part of a multi-detector plan (from ants_autotune_multi),
  // valid for the grid configuration whose hash is mplan_key
  uint64_t mplan_key = 0;
  int32_t mplan_T = 0, mplan_lds = 1, mplan_bpc = 0;
  // workspace of the LRF fit (per-wave partial normal equations)
  void* ws_fit = nullptr;
  size_t ws_fit_bytes = 0;
  void* ws_fit2 = nullptr;       // two-dimensional LRF fits
  size_t ws_fit2_bytes = 0;
};
