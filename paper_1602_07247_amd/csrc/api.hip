// Host side of the C ABI declared in include/ants.h: argument checking,
// LRF-set upload (FP32 piecewise-polynomial tables for the screening pass,
// FP64 B-spline coefficients for decisions and outputs) and kernel launch.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "ants_internal.h"

using ants::DevLrf;
using ants::GenP;
using ants::GridP;
using ants::IoP;
using ants::kMaxNodes;
using ants::kMaxSensors;

namespace {

thread_local std::string g_err;

// B-spline coefficients c[m..m+3] of one interval -> polynomial in t
void to_poly(const double* c, double out[4]) {
  out[0] = (c[0] + 4.0 * c[1] + c[2]) / 6.0;
  out[1] = (c[2] - c[0]) / 2.0;
  out[2] = (c[0] - 2.0 * c[1] + c[2]) / 2.0;
  out[3] = (-c[0] + 3.0 * c[1] - 3.0 * c[2] + c[3]) / 6.0;
}

template <class T>
hipError_t upload(T** dst, const T* src, size_t n) {
  *dst = nullptr;
  if (n == 0) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, n * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
}

int g_num_cu = 0;

// ---- LRF-set file (see ants_lrf_write in ants.h)
constexpr char kLrfMagic[8] = {'A', 'N', 'T', 'S', 'L', 'R', 'F', '1'};
constexpr size_t kLrfHeader = 8 + 6 * 4 + 4 * 8 + 8;   // magic, ints, domain, n_coef

uint64_t fnv1a(const unsigned char* p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

size_t coef_count(int kind, int shared, int ns, int nb0, int nb1) {
  const size_t nc0 = (size_t)nb0 + 2, nc1 = kind == ANTS_LRF_AXIAL ? 1 : (size_t)nb1 + 2;
  return nc0 * nc1 * (shared ? 1 : (size_t)ns);
}

size_t pad8(size_t n) { return (n + 7) & ~(size_t)7; }

// file size for a header's counts (0 when they are out of range)
size_t lrf_file_bytes(int ns, size_t ncoef) {
  return kLrfHeader + 8 * 3 * (size_t)ns + pad8((size_t)ns) + 8 * ncoef + 8;
}

template <class T>
void put(std::vector<unsigned char>& b, const T& v) {
  const unsigned char* p = (const unsigned char*)&v;
  b.insert(b.end(), p, p + sizeof(T));
}
template <class T>
T get(const unsigned char*& p) {
  T v;
  memcpy(&v, p, sizeof(T));
  p += sizeof(T);
  return v;
}

ants_status write_lrf_file(const char* path, int ns, int kind, int shared, const int32_t nk[2],
                           const double lo[2], const double hi[2], const double* xy,
                           const double* gain, const uint8_t* active, const double* coef,
                           size_t ncoef) {
  std::vector<unsigned char> b;
  b.reserve(lrf_file_bytes(ns, ncoef));
  b.insert(b.end(), kLrfMagic, kLrfMagic + 8);
  put<int32_t>(b, ns);
  put<int32_t>(b, kind);
  put<int32_t>(b, shared);
  put<int32_t>(b, nk[0]);
  put<int32_t>(b, nk[1]);
  put<int32_t>(b, 0);
  for (int a = 0; a < 2; ++a) put<double>(b, lo[a]);
  for (int a = 0; a < 2; ++a) put<double>(b, hi[a]);
  put<int64_t>(b, (int64_t)ncoef);
  for (int i = 0; i < 2 * ns; ++i) put<double>(b, xy[i]);
  for (int i = 0; i < ns; ++i) put<double>(b, gain ? gain[i] : 1.0);
  for (int i = 0; i < ns; ++i) b.push_back(active ? (active[i] ? 1 : 0) : 1);
  while (b.size() % 8) b.push_back(0);
  for (size_t i = 0; i < ncoef; ++i) put<double>(b, coef[i]);
  put<uint64_t>(b, fnv1a(b.data(), b.size()));
  FILE* f = fopen(path, "wb");
  if (!f) return ants::set_error(ANTS_E_ARG, "cannot open %s for writing", path);
  const bool ok = fwrite(b.data(), 1, b.size(), f) == b.size();
  const bool closed = fclose(f) == 0;
  if (!ok || !closed) return ants::set_error(ANTS_E_ARG, "writing %s failed", path);
  return ANTS_OK;
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void copy_i32_kernel(const int32_t* a, int32_t* b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace

namespace ants {

ants_status set_error(ants_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

ants_status hip_error(hipError_t e, const char* what) {
  return set_error(e == hipErrorOutOfMemory ? ANTS_E_NOMEM : ANTS_E_DEVICE, "%s: %s", what,
                   hipGetErrorString(e));
}

int num_cu() {
  if (g_num_cu == 0) {
    int dev = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess ||
        g_num_cu <= 0)
      g_num_cu = 256;
  }
  return g_num_cu;
}

hipError_t ensure(void** p, size_t* have, size_t need) {
  if (*p && *have >= need) return hipSuccess;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *have = 0;
  hipError_t e = hipMalloc(p, need);
  if (e == hipSuccess) *have = need;
  return e;
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t launch_copy_i32(const int32_t* a, int32_t* b, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, b, n);
  return hipGetLastError();
}

uint64_t grid_cfg_key(const ants_grid_cfg& c) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
      h ^= b[i];
      h *= 1099511628211ull;
    }
  };
  mix(c.nodes, sizeof(c.nodes));
  mix(&c.iterations, sizeof(c.iterations));
  mix(&c.stat, sizeof(c.stat));
  mix(&c.start, sizeof(c.start));
  mix(&c.screen_scale, sizeof(c.screen_scale));
  mix(&c.seed_steps, sizeof(c.seed_steps));
  mix(&c.cut_signal, sizeof(c.cut_signal));
  mix(&c.cut_distance, sizeof(c.cut_distance));
  return h | 1;
}

void apply_grid_plan(const ants_lrfset* S, const ants_grid_cfg* cfg, GridP* G) {
  const uint64_t k = grid_cfg_key(*cfg);
  for (int i = 0; i < S->n_gplan; ++i)
    if (S->gplan[i].key == k) {
      G->plan_wpb = S->gplan[i].wpb;
      G->plan_bpc = S->gplan[i].bpc;
      G->plan_screen = S->gplan[i].screen;
      return;
    }
}

ants_status grid_params(const DevLrf& L, const ants_grid_cfg* cfg, GridP* Gp) {
  GridP& G = *Gp;
  memset(&G, 0, sizeof(G));
  G.fb_thr = -1.0;   // no fallback list unless the seeded path sets a threshold
  G.nx = cfg->nodes[0];
  G.ny = cfg->nodes[1];
  G.nz = cfg->nodes[2];
  for (int a = 0; a < 3; ++a)
    if (cfg->nodes[a] < 1 || cfg->nodes[a] % 2 == 0)
      return set_error(ANTS_E_ARG, "nodes[%d] = %d must be odd and >= 1", a, cfg->nodes[a]);
  if ((int64_t)G.nx * G.ny * G.nz > kMaxNodes)
    return set_error(ANTS_E_ARG, "grid of %d x %d x %d exceeds %d nodes", G.nx, G.ny, G.nz,
                     kMaxNodes);
  if (L.kind != ANTS_LRF_RZ && L.kind != ANTS_LRF_SLICED && G.nz != 1)
    return set_error(ANTS_E_ARG, "a 2-D LRF needs nodes[2] = 1");
  if (G.nz > 101) return set_error(ANTS_E_ARG, "nodes[2] = %d exceeds 101", G.nz);
  G.nn = G.nx * G.ny * G.nz;
  G.hx = (G.nx - 1) / 2;
  G.hy = (G.ny - 1) / 2;
  G.hz = (G.nz - 1) / 2;
  {
    // bits per axis index; at most 12 in total for grids of <= 512 nodes
    auto bits = [](int n) { int b = 0; while ((1 << b) < n) ++b; return b; };
    const int bx = bits(G.nx), by = bits(G.ny);
    G.shy = bx;
    G.shz = bx + by;
    G.mskx = (1 << bx) - 1;
    G.msky = (1 << by) - 1;
  }
  G.K = cfg->iterations;
  if (G.K < 0 || G.K > 64) return set_error(ANTS_E_ARG, "iterations = %d outside 0..64", G.K);
  if (!(cfg->shrink > 0.0 && cfg->shrink <= 1.0))
    return set_error(ANTS_E_ARG, "shrink = %g outside (0, 1]", cfg->shrink);
  for (int a = 0; a < 3; ++a)
    if (cfg->nodes[a] > 1 && !(cfg->step0[a] > 0.0 && isfinite(cfg->step0[a])))
      return set_error(ANTS_E_ARG, "step0[%d] = %g must be positive", a, cfg->step0[a]);
  if (!(cfg->l_floor > 0.0) || !(cfg->v_floor > 0.0))
    return set_error(ANTS_E_ARG, "l_floor and v_floor must be positive");
  if (cfg->stat != ANTS_STAT_ML && cfg->stat != ANTS_STAT_CHI2)
    return set_error(ANTS_E_ARG, "unknown statistic %d", cfg->stat);
  if (cfg->start < ANTS_START_COG || cfg->start > ANTS_START_SEED)
    return set_error(ANTS_E_ARG, "unknown start option %d", cfg->start);
  if (!(cfg->screen_scale == 0.0 || cfg->screen_scale >= 1.0))
    return set_error(ANTS_E_ARG, "screen_scale = %g must be 0 or >= 1", cfg->screen_scale);
  if (!isfinite(cfg->z_start)) return set_error(ANTS_E_ARG, "z_start not finite");
  G.dim = G.nz > 1 ? 3 : 2;
  G.stat = cfg->stat;
  G.start = cfg->start;
  G.shrink = cfg->shrink;
  G.s0x = G.nx > 1 ? cfg->step0[0] : 0.0;
  G.s0y = G.ny > 1 ? cfg->step0[1] : 0.0;
  G.s0z = G.nz > 1 ? cfg->step0[2] : 0.0;
  G.z_start = cfg->z_start;
  G.lfloor = cfg->l_floor;
  G.vfloor = cfg->v_floor;
  double sc = cfg->screen_scale == 0.0 ? 1.0 : cfg->screen_scale;
  G.margin_scale = sc > 3e38 ? 3e38f : (float)sc;
  if (!(cfg->cut_signal >= 0.0 && cfg->cut_signal < 1e300) ||
      !(cfg->cut_distance >= 0.0 && cfg->cut_distance < 1e300))
    return set_error(ANTS_E_ARG, "cut_signal = %g / cut_distance = %g must be finite and >= 0",
                     cfg->cut_signal, cfg->cut_distance);
  G.cut_signal = cfg->cut_signal;
  G.cut_dist = cfg->cut_distance;
  G.seed_steps = 0;
  if (cfg->start == ANTS_START_SEED && cfg->seed_steps) {
    if (!(cfg->seed_kmin >= 1 && cfg->seed_kmin <= cfg->seed_kmax && cfg->seed_kmax <= G.K &&
          cfg->seed_kmax <= kMaxSeedSteps))
      return set_error(ANTS_E_ARG,
                       "need 1 <= seed_kmin (%d) <= seed_kmax (%d) <= min(iterations (%d), %d)",
                       cfg->seed_kmin, cfg->seed_kmax, G.K, kMaxSeedSteps);
    if (!(cfg->seed_kappa > 0.0 && isfinite(cfg->seed_kappa)))
      return set_error(ANTS_E_ARG, "seed_kappa = %g must be positive", cfg->seed_kappa);
    for (int a = 0; a < 3; ++a)
      if (!(cfg->seed_scale[a] >= 0.0 && isfinite(cfg->seed_scale[a])))
        return set_error(ANTS_E_ARG, "seed_scale[%d] = %g invalid", a, cfg->seed_scale[a]);
    G.seed_steps = 1;
    G.kappa = cfg->seed_kappa;
    G.kmin = cfg->seed_kmin;
    G.kmax = cfg->seed_kmax;
    const double s0[3] = {G.s0x, G.s0y, G.s0z};
    for (int a = 0; a < 3; ++a) {
      G.sscale[a] = cfg->seed_scale[a];
      double f = s0[a];
      for (int k = 1; k < G.K; ++k) f *= cfg->shrink;
      G.sfinal[a] = f;
    }
  }
  return ANTS_OK;
}

}  // namespace ants

using ants::set_error;
#define fail set_error
#define hip_fail ants::hip_error

extern "C" {

const char* ants_last_error(void) { return g_err.c_str(); }
const char* ants_version(void) { return "ants-mi355x 0.1 (gfx950)"; }

ants_status ants_lrfset_destroy(ants_lrfset* set) {
  if (!set) return ANTS_OK;
  for (void* p : set->allocs) (void)hipFree(p);
  if (set->ws_seeds) (void)hipFree(set->ws_seeds);
  if (set->ws_list) (void)hipFree(set->ws_list);
  if (set->ws_count) (void)hipFree(set->ws_count);
  if (set->ws_multi) (void)hipFree(set->ws_multi);
  if (set->ms_copied) {
    (void)hipEventSynchronize(set->ms_copied);
    (void)hipEventDestroy(set->ms_copied);
  }
  if (set->ms_host) (void)hipHostFree(set->ms_host);
  if (set->ws_fit) (void)hipFree(set->ws_fit);
  if (set->ws_fit2) (void)hipFree(set->ws_fit2);
  delete set;
  return ANTS_OK;
}

ants_status ants_lrfset_info(const ants_lrfset* set, int32_t* n_sensors, int32_t* n_active,
                             int32_t* kind) {
  if (!set) return fail(ANTS_E_ARG, "ants_lrfset_info: NULL set");
  if (n_sensors) *n_sensors = set->ns;
  if (n_active) *n_active = set->d.na;
  if (kind) *kind = set->d.kind;
  return ANTS_OK;
}

ants_status ants_lrfset_create(const ants_lrf_desc* D, ants_lrfset** out) {
  if (!out) return fail(ANTS_E_ARG, "ants_lrfset_create: NULL out");
  *out = nullptr;
  if (!D) return fail(ANTS_E_ARG, "ants_lrfset_create: NULL descriptor");
  const int ns = D->n_sensors;
  if (ns < 1 || ns > kMaxSensors)
    return fail(ANTS_E_ARG, "n_sensors = %d outside 1..%d", ns, kMaxSensors);
  if (!D->sensor_xy || !D->coef) return fail(ANTS_E_ARG, "sensor_xy and coef are required");
  const int kind = D->kind;
  if (kind < ANTS_LRF_AXIAL || kind > ANTS_LRF_SLICED)
    return fail(ANTS_E_ARG, "unknown LRF kind %d", kind);
  const bool one_axis = kind == ANTS_LRF_AXIAL || kind == ANTS_LRF_COMPOSITE;
  const int nb0 = D->n_knots[0];
  const int nb1 = one_axis ? 1 : D->n_knots[1];
  if (nb0 < 2 || nb0 > 256 || (!one_axis && (nb1 < 2 || nb1 > 256)))
    return fail(ANTS_E_ARG, "n_knots (%d, %d) outside 2..256", D->n_knots[0], D->n_knots[1]);
  const int naxes = one_axis ? 1 : 2;
  for (int a = 0; a < naxes; ++a)
    if (!(isfinite(D->lo[a]) && isfinite(D->hi[a]) && D->lo[a] < D->hi[a]))
      return fail(ANTS_E_FORMAT, "axis %d domain [%g, %g] invalid", a, D->lo[a], D->hi[a]);
  if (kind != ANTS_LRF_XY && kind != ANTS_LRF_SLICED && D->lo[0] != 0.0)
    return fail(ANTS_E_UNSUPPORTED, "the r axis must start at 0 (lo[0] = %g)", D->lo[0]);
  if ((kind == ANTS_LRF_RZ || kind == ANTS_LRF_COMPOSITE) && !D->shared)
    return fail(ANTS_E_UNSUPPORTED, "r-z LRFs and the axial part of composite LRFs must be "
                                    "shared by all sensors");
  // composite: the XY residual
  const int xnb0 = kind == ANTS_LRF_COMPOSITE ? D->xy_knots[0] : 0;
  const int xnb1 = kind == ANTS_LRF_COMPOSITE ? D->xy_knots[1] : 0;
  const int xntab = kind == ANTS_LRF_COMPOSITE ? (D->xy_shared ? 1 : ns) : 0;
  const size_t xper = (size_t)(xnb0 + 2) * (xnb1 + 2);
  if (kind == ANTS_LRF_COMPOSITE) {
    if (xnb0 < 2 || xnb0 > 256 || xnb1 < 2 || xnb1 > 256)
      return fail(ANTS_E_ARG, "xy_knots (%d, %d) outside 2..256", xnb0, xnb1);
    if (!D->xy_coef) return fail(ANTS_E_ARG, "a composite LRF needs xy_coef");
    for (int a = 0; a < 2; ++a)
      if (!(isfinite(D->xy_lo[a]) && isfinite(D->xy_hi[a]) && D->xy_lo[a] < D->xy_hi[a]))
        return fail(ANTS_E_FORMAT, "residual axis %d domain [%g, %g] invalid", a, D->xy_lo[a],
                    D->xy_hi[a]);
    for (size_t i = 0; i < xper * xntab; ++i)
      if (!isfinite(D->xy_coef[i])) return fail(ANTS_E_FORMAT, "xy_coef[%zu] is not finite", i);
  }
  // sliced: the z planes
  const int np = kind == ANTS_LRF_SLICED ? D->n_planes : 1;
  if (kind == ANTS_LRF_SLICED) {
    if (np < 2 || np > 64) return fail(ANTS_E_ARG, "n_planes = %d outside 2..64", np);
    if (!(isfinite(D->z_lo) && isfinite(D->z_hi) && D->z_lo < D->z_hi))
      return fail(ANTS_E_FORMAT, "plane range [%g, %g] invalid", D->z_lo, D->z_hi);
  }
  const int nc0 = nb0 + 2, nc1 = one_axis ? 1 : nb1 + 2;
  const int ntab = D->shared ? 1 : ns;
  const size_t per = (size_t)nc0 * nc1 * np;
  for (size_t i = 0; i < per * ntab; ++i)
    if (!isfinite(D->coef[i])) return fail(ANTS_E_FORMAT, "coef[%zu] is not finite", i);
  for (int i = 0; i < 2 * ns; ++i)
    if (!isfinite(D->sensor_xy[i])) return fail(ANTS_E_FORMAT, "sensor_xy[%d] not finite", i);
  if (D->gain)
    for (int i = 0; i < ns; ++i)
      if (!(D->gain[i] > 0.0 && isfinite(D->gain[i])))
        return fail(ANTS_E_FORMAT, "gain[%d] = %g must be positive", i, D->gain[i]);

  // active sensors in their original order
  std::vector<int32_t> col, tab, xtab;
  std::vector<double> X, Y, g;
  for (int i = 0; i < ns; ++i) {
    if (D->active && !D->active[i]) continue;
    col.push_back(i);
    tab.push_back(D->shared ? 0 : i);
    xtab.push_back(D->xy_shared ? 0 : i);
    X.push_back(D->sensor_xy[2 * i]);
    Y.push_back(D->sensor_xy[2 * i + 1]);
    g.push_back(D->gain ? D->gain[i] : 1.0);
  }
  const int na = (int)col.size();

  const int nint0 = nb0 - 1;
  const int nintp = nint0 + 1;  // one all-zero interval past the domain end
  std::vector<float> pp, c32, xc32;
  if (kind == ANTS_LRF_AXIAL || kind == ANTS_LRF_RZ || kind == ANTS_LRF_COMPOSITE) {
    const int rows = kind == ANTS_LRF_RZ ? nc1 : ntab;
    pp.assign((size_t)rows * nintp * 4, 0.f);
    for (int r = 0; r < rows; ++r)
      for (int m = 0; m < nint0; ++m) {
        double p[4];
        to_poly(D->coef + (size_t)r * nc0 + m, p);
        for (int k = 0; k < 4; ++k) pp[((size_t)r * nintp + m) * 4 + k] = (float)p[k];
      }
    if (kind == ANTS_LRF_AXIAL && (size_t)ntab * nintp * 16 > 48 * 1024)
      return fail(ANTS_E_UNSUPPORTED, "per-sensor axial tables exceed 48 KiB of LDS");
  } else {
    c32.resize(per * ntab);
    for (size_t i = 0; i < c32.size(); ++i) c32[i] = (float)D->coef[i];
  }
  if (kind == ANTS_LRF_COMPOSITE) {
    xc32.resize(xper * xntab);
    for (size_t i = 0; i < xc32.size(); ++i) xc32[i] = (float)D->xy_coef[i];
  }

  ants_lrfset* S = new ants_lrfset();
  hipGetDevice(&S->device);
  S->ns = ns;
  DevLrf& d = S->d;
  memset(&d, 0, sizeof(d));
  d.kind = kind;
  d.shared = D->shared ? 1 : 0;
  d.ns = ns;
  d.na = na;
  d.nb0 = nb0;
  d.nb1 = nb1;
  d.nc0 = nc0;
  d.nc1 = nc1;
  d.nintp = nintp;
  d.ntab = ntab;
  d.lo0 = D->lo[0];
  d.hi0 = D->hi[0];
  d.lo1 = one_axis ? 0.0 : D->lo[1];
  d.hi1 = one_axis ? 1.0 : D->hi[1];
  d.d0 = (d.hi0 - d.lo0) / (nb0 - 1);
  d.d1 = one_axis ? 1.0 : (d.hi1 - d.lo1) / (nb1 - 1);
  if (kind == ANTS_LRF_COMPOSITE) {
    d.xnb0 = xnb0;
    d.xnb1 = xnb1;
    d.xnc0 = xnb0 + 2;
    d.xnc1 = xnb1 + 2;
    d.xlo0 = D->xy_lo[0];
    d.xhi0 = D->xy_hi[0];
    d.xlo1 = D->xy_lo[1];
    d.xhi1 = D->xy_hi[1];
    d.xinv_d0 = (xnb0 - 1) / (d.xhi0 - d.xlo0);
    d.xinv_d1 = (xnb1 - 1) / (d.xhi1 - d.xlo1);
  }
  if (kind == ANTS_LRF_SLICED) {
    d.nplanes = np;
    d.zlo = D->z_lo;
    d.zhi = D->z_hi;
    d.inv_dz = (np - 1) / (D->z_hi - D->z_lo);
  }
  d.finv0 = (float)(1.0 / d.d0);
  d.inv_d0 = 1.0 / d.d0;
  d.inv_d1 = 1.0 / d.d1;
  // non-negative pieces: the screen can skip the clamp at 0
  d.nonneg = 0;
  if (!pp.empty() && kind != ANTS_LRF_COMPOSITE) {
    bool nn = true;
    for (size_t r = 0; r + 3 < pp.size() && nn; r += 4) {
      const double a0 = pp[r], a1 = pp[r + 1], a2 = pp[r + 2], a3 = pp[r + 3];
      auto val = [&](double t) { return a0 + t * (a1 + t * (a2 + t * a3)); };
      double mn = fmin(val(0.0), val(1.0));
      // stationary points of the cubic in (0, 1)
      const double A = 3.0 * a3, B = 2.0 * a2, Cc = a1;
      if (A != 0.0) {
        const double disc = B * B - 4.0 * A * Cc;
        if (disc >= 0.0) {
          const double sq = sqrt(disc);
          const double t1 = (-B - sq) / (2.0 * A), t2 = (-B + sq) / (2.0 * A);
          if (t1 > 0.0 && t1 < 1.0) mn = fmin(mn, val(t1));
          if (t2 > 0.0 && t2 < 1.0) mn = fmin(mn, val(t2));
        }
      } else if (B != 0.0) {
        const double t1 = -Cc / B;
        if (t1 > 0.0 && t1 < 1.0) mn = fmin(mn, val(t1));
      }
      nn = mn >= 0.0;
    }
    d.nonneg = nn ? 1 : 0;
  }

  hipError_t e = hipSuccess;
  int32_t *dcol = nullptr, *dtab = nullptr;
  double *dX = nullptr, *dY = nullptr, *dg = nullptr, *dc64 = nullptr;
  float *dpp = nullptr, *dc32 = nullptr;
  if (e == hipSuccess) e = upload(&dcol, col.data(), col.size());
  if (dcol) S->allocs.push_back(dcol);
  if (e == hipSuccess) e = upload(&dtab, tab.data(), tab.size());
  if (dtab) S->allocs.push_back(dtab);
  if (e == hipSuccess) e = upload(&dX, X.data(), X.size());
  if (dX) S->allocs.push_back(dX);
  if (e == hipSuccess) e = upload(&dY, Y.data(), Y.size());
  if (dY) S->allocs.push_back(dY);
  if (e == hipSuccess) e = upload(&dg, g.data(), g.size());
  if (dg) S->allocs.push_back(dg);
  if (e == hipSuccess) e = upload(&dc64, D->coef, per * ntab);
  if (dc64) S->allocs.push_back(dc64);
  if (e == hipSuccess) e = upload(&dpp, pp.data(), pp.size());
  if (dpp) S->allocs.push_back(dpp);
  if (e == hipSuccess) e = upload(&dc32, c32.data(), c32.size());
  if (dc32) S->allocs.push_back(dc32);
  int32_t* dxtab = nullptr;
  float* dxc32 = nullptr;
  double* dxc64 = nullptr;
  if (kind == ANTS_LRF_COMPOSITE) {
    if (e == hipSuccess) e = upload(&dxtab, xtab.data(), xtab.size());
    if (dxtab) S->allocs.push_back(dxtab);
    if (e == hipSuccess) e = upload(&dxc32, xc32.data(), xc32.size());
    if (dxc32) S->allocs.push_back(dxc32);
    if (e == hipSuccess) e = upload(&dxc64, D->xy_coef, xper * xntab);
    if (dxc64) S->allocs.push_back(dxc64);
  }
  if (e != hipSuccess) {
    ants_lrfset_destroy(S);
    return hip_fail(e, "ants_lrfset_create upload");
  }
  S->h_kind = kind;
  S->h_shared = D->shared ? 1 : 0;
  S->h_knots[0] = D->n_knots[0];
  S->h_knots[1] = kind == ANTS_LRF_AXIAL ? 0 : D->n_knots[1];
  for (int a = 0; a < 2; ++a) {
    S->h_lo[a] = a < naxes ? D->lo[a] : 0.0;
    S->h_hi[a] = a < naxes ? D->hi[a] : 0.0;
  }
  S->h_xy.assign(D->sensor_xy, D->sensor_xy + 2 * ns);
  S->h_gain.resize(ns);
  S->h_active.resize(ns);
  for (int i = 0; i < ns; ++i) {
    S->h_gain[i] = D->gain ? D->gain[i] : 1.0;
    S->h_active[i] = (!D->active || D->active[i]) ? 1 : 0;
  }
  S->h_coef.assign(D->coef, D->coef + per * ntab);
  d.col = dcol;
  d.tab = dtab;
  d.X = dX;
  d.Y = dY;
  d.g = dg;
  d.pp = dpp;
  d.c32 = dc32;
  d.c64 = dc64;
  d.xtab = dxtab;
  d.xc32 = dxc32;
  d.xc64 = dxc64;
  *out = S;
  return ANTS_OK;
}

ants_status ants_lrf_write(const ants_lrf_desc* D, const char* path) {
  if (!D || !path) return fail(ANTS_E_ARG, "ants_lrf_write: NULL descriptor or path");
  const int ns = D->n_sensors;
  if (ns < 1 || ns > kMaxSensors)
    return fail(ANTS_E_ARG, "n_sensors = %d outside 1..%d", ns, kMaxSensors);
  if (!D->sensor_xy || !D->coef) return fail(ANTS_E_ARG, "sensor_xy and coef are required");
  if (D->kind == ANTS_LRF_COMPOSITE || D->kind == ANTS_LRF_SLICED)
    return fail(ANTS_E_UNSUPPORTED, "composite and sliced sets have no file format");
  if (D->kind != ANTS_LRF_AXIAL && D->kind != ANTS_LRF_XY && D->kind != ANTS_LRF_RZ)
    return fail(ANTS_E_ARG, "unknown LRF kind %d", D->kind);
  const int nb1 = D->kind == ANTS_LRF_AXIAL ? 0 : D->n_knots[1];
  if (D->n_knots[0] < 2 || D->n_knots[0] > 256 ||
      (D->kind != ANTS_LRF_AXIAL && (nb1 < 2 || nb1 > 256)))
    return fail(ANTS_E_ARG, "n_knots (%d, %d) outside 2..256", D->n_knots[0], D->n_knots[1]);
  const int32_t nk[2] = {D->n_knots[0], nb1};
  const double lo[2] = {D->lo[0], D->kind == ANTS_LRF_AXIAL ? 0.0 : D->lo[1]};
  const double hi[2] = {D->hi[0], D->kind == ANTS_LRF_AXIAL ? 0.0 : D->hi[1]};
  return write_lrf_file(path, ns, D->kind, D->shared ? 1 : 0, nk, lo, hi, D->sensor_xy, D->gain,
                        D->active, D->coef,
                        coef_count(D->kind, D->shared, ns, D->n_knots[0], nb1));
}

ants_status ants_lrfset_save(const ants_lrfset* S, const char* path) {
  if (!S || !path) return fail(ANTS_E_ARG, "ants_lrfset_save: NULL set or path");
  if (S->h_kind == ANTS_LRF_COMPOSITE || S->h_kind == ANTS_LRF_SLICED)
    return fail(ANTS_E_UNSUPPORTED, "composite and sliced sets have no file format");
  return write_lrf_file(path, S->ns, S->h_kind, S->h_shared, S->h_knots, S->h_lo, S->h_hi,
                        S->h_xy.data(), S->h_gain.data(), S->h_active.data(), S->h_coef.data(),
                        S->h_coef.size());
}

ants_status ants_lrfset_load(const char* path, ants_lrfset** out) {
  if (!out) return fail(ANTS_E_ARG, "ants_lrfset_load: NULL out");
  *out = nullptr;
  if (!path) return fail(ANTS_E_ARG, "ants_lrfset_load: NULL path");
  FILE* f = fopen(path, "rb");
  if (!f) return fail(ANTS_E_ARG, "cannot open %s", path);
  std::vector<unsigned char> b;
  unsigned char buf[65536];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) {
    b.insert(b.end(), buf, buf + got);
    if (b.size() > ((size_t)1 << 30)) break;
  }
  fclose(f);
  if (b.size() < kLrfHeader + 8) return fail(ANTS_E_FORMAT, "%s is truncated", path);
  if (memcmp(b.data(), kLrfMagic, 8) != 0)
    return fail(ANTS_E_FORMAT, "%s is not an LRF-set file (magic)", path);
  const unsigned char* p = b.data() + 8;
  const int32_t ns = get<int32_t>(p), kind = get<int32_t>(p), shared = get<int32_t>(p);
  int32_t nk[2];
  nk[0] = get<int32_t>(p);
  nk[1] = get<int32_t>(p);
  (void)get<int32_t>(p);
  double lo[2], hi[2];
  for (int a = 0; a < 2; ++a) lo[a] = get<double>(p);
  for (int a = 0; a < 2; ++a) hi[a] = get<double>(p);
  const int64_t ncoef = get<int64_t>(p);
  if (ns < 1 || ns > kMaxSensors || (kind != ANTS_LRF_AXIAL && kind != ANTS_LRF_XY &&
                                     kind != ANTS_LRF_RZ) ||
      (shared != 0 && shared != 1) || nk[0] < 2 || nk[0] > 256 ||
      (kind != ANTS_LRF_AXIAL && (nk[1] < 2 || nk[1] > 256)))
    return fail(ANTS_E_FORMAT, "%s: header out of range", path);
  if (ncoef != (int64_t)coef_count(kind, shared, ns, nk[0], nk[1]))
    return fail(ANTS_E_FORMAT, "%s: coefficient count %lld does not match the header", path,
                (long long)ncoef);
  if (b.size() != lrf_file_bytes(ns, (size_t)ncoef))
    return fail(ANTS_E_FORMAT, "%s: %zu bytes, expected %zu (truncated or extended)", path,
                b.size(), lrf_file_bytes(ns, (size_t)ncoef));
  uint64_t sum;
  memcpy(&sum, b.data() + b.size() - 8, 8);
  if (sum != fnv1a(b.data(), b.size() - 8))
    return fail(ANTS_E_FORMAT, "%s: checksum mismatch", path);
  std::vector<double> xy(2 * (size_t)ns), gain(ns), coef((size_t)ncoef);
  std::vector<uint8_t> active(ns);
  memcpy(xy.data(), p, 16 * (size_t)ns);
  p += 16 * (size_t)ns;
  memcpy(gain.data(), p, 8 * (size_t)ns);
  p += 8 * (size_t)ns;
  memcpy(active.data(), p, (size_t)ns);
  p += pad8((size_t)ns);
  memcpy(coef.data(), p, 8 * (size_t)ncoef);
  ants_lrf_desc D;
  memset(&D, 0, sizeof(D));
  D.n_sensors = ns;
  D.sensor_xy = xy.data();
  D.gain = gain.data();
  D.active = active.data();
  D.kind = kind;
  D.shared = shared;
  D.n_knots[0] = nk[0];
  D.n_knots[1] = kind == ANTS_LRF_AXIAL ? 1 : nk[1];
  for (int a = 0; a < 2; ++a) {
    D.lo[a] = lo[a];
    D.hi[a] = hi[a];
  }
  if (kind == ANTS_LRF_AXIAL) {
    D.lo[1] = 0.0;
    D.hi[1] = 1.0;
  }
  D.coef = coef.data();
  return ants_lrfset_create(&D, out);
}

ants_status ants_reconstruct(ants_lrfset* set, const ants_grid_cfg* cfg, int64_t n_events,
                             const float* d_signals, const float* d_seeds, ants_out out,
                             void* hip_stream) {
  if (!set || !cfg) return fail(ANTS_E_ARG, "ants_reconstruct: NULL set or cfg");
  if (n_events < 0) return fail(ANTS_E_ARG, "n_events = %lld < 0", (long long)n_events);
  if (n_events > ((int64_t)1 << 31) - 1)
    return fail(ANTS_E_ARG, "n_events = %lld exceeds 2^31-1", (long long)n_events);
  const DevLrf& L = set->d;
  GridP G;
  ants_status st = ants::grid_params(L, cfg, &G);
  if (st != ANTS_OK) return st;
  ants::apply_grid_plan(set, cfg, &G);
  if (cfg->start == ANTS_START_SEED && !d_seeds)
    return fail(ANTS_E_ARG, "start = SEED needs d_seeds");
  if (n_events == 0) return ANTS_OK;
  if (!d_signals) return fail(ANTS_E_ARG, "d_signals is NULL");
  if (!out.x || !out.y || !out.z || !out.E || !out.lnl || !out.chi2 || !out.ndf || !out.status)
    return fail(ANTS_E_ARG, "an ants_out field other than path/n_fp64 is NULL");

  IoP io;
  memset(&io, 0, sizeof(io));
  io.sig = d_signals;
  io.ld = set->ns;
  io.seeds = d_seeds;
  io.x = out.x;
  io.y = out.y;
  io.z = out.z;
  io.E = out.E;
  io.lnl = out.lnl;
  io.chi2 = out.chi2;
  io.ndf = out.ndf;
  io.status = out.status;
  io.path = out.path;
  io.nfp = out.n_fp64;
  io.n = n_events;

  int dev = 0;
  hipGetDevice(&dev);
  if (dev != set->device)
    return fail(ANTS_E_ARG, "LRF set lives on device %d, current device is %d", set->device,
                dev);
  hipError_t e = ants::launch_grid(L, G, io, (hipStream_t)hip_stream, ants::num_cu() * 8);
  if (e != hipSuccess) return hip_fail(e, "ants_reconstruct launch");
  return ANTS_OK;
}

ants_status ants_set_plan(ants_lrfset* set, const ants_grid_cfg* cfg,
                          const ants_grid_plan* plan) {
  if (!set || !cfg) return fail(ANTS_E_ARG, "ants_set_plan: NULL set or cfg");
  const uint64_t k = ants::grid_cfg_key(*cfg);
  int slot = -1;
  for (int i = 0; i < set->n_gplan; ++i)
    if (set->gplan[i].key == k) slot = i;
  if (!plan) {   // remove
    if (slot >= 0) {
      for (int i = slot + 1; i < set->n_gplan; ++i) set->gplan[i - 1] = set->gplan[i];
      --set->n_gplan;
    }
    return ANTS_OK;
  }
  if (plan->waves_per_block != 1 && plan->waves_per_block != 2 && plan->waves_per_block != 4)
    return fail(ANTS_E_ARG, "waves_per_block = %d must be 1, 2 or 4", plan->waves_per_block);
  if (plan->blocks_per_cu < 0 || plan->blocks_per_cu > 32)
    return fail(ANTS_E_ARG, "blocks_per_cu = %d outside 0..32", plan->blocks_per_cu);
  if (plan->screen != 0 && plan->screen != 1)
    return fail(ANTS_E_ARG, "screen = %d must be 0 or 1", plan->screen);
  if (slot < 0) {
    if (set->n_gplan == 8) {   // full: drop the oldest
      for (int i = 1; i < 8; ++i) set->gplan[i - 1] = set->gplan[i];
      set->n_gplan = 7;
    }
    slot = set->n_gplan++;
  }
  set->gplan[slot] = {k, plan->waves_per_block, plan->blocks_per_cu, plan->screen};
  return ANTS_OK;
}

ants_status ants_autotune(ants_lrfset* set, const ants_grid_cfg* cfg, int64_t n_sample,
                          const float* d_signals, const float* d_seeds, ants_out scratch,
                          ants_grid_plan* best, double* host_ms, void* hip_stream) {
  if (!set || !cfg || !best) return fail(ANTS_E_ARG, "ants_autotune: NULL set, cfg or best");
  if (n_sample < 1 || n_sample > ((int64_t)1 << 31) - 1)
    return fail(ANTS_E_ARG, "n_sample = %lld out of range", (long long)n_sample);
  GridP G;
  ants_status st = ants::grid_params(set->d, cfg, &G);
  if (st != ANTS_OK) return st;
  if (cfg->start == ANTS_START_SEED && !d_seeds)
    return fail(ANTS_E_ARG, "start = SEED needs d_seeds");
  if (!d_signals || !scratch.x || !scratch.y || !scratch.z || !scratch.E || !scratch.lnl ||
      !scratch.chi2 || !scratch.ndf || !scratch.status)
    return fail(ANTS_E_ARG, "NULL signals or scratch output");
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev != set->device) return fail(ANTS_E_ARG, "LRF set lives on another device");
  IoP io;
  memset(&io, 0, sizeof(io));
  io.sig = d_signals;
  io.ld = set->ns;
  io.seeds = d_seeds;
  io.x = scratch.x;
  io.y = scratch.y;
  io.z = scratch.z;
  io.E = scratch.E;
  io.lnl = scratch.lnl;
  io.chi2 = scratch.chi2;
  io.ndf = scratch.ndf;
  io.status = scratch.status;
  io.n = n_sample;
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return fail(ANTS_E_DEVICE, "hipEventCreate failed");
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(ANTS_E_DEVICE, "hipEventCreate failed");
  }
  // candidates: screen variant (where the column-factored one applies),
  // waves per block, cap on blocks per CU; the kernel alone is timed
  const bool fact = (set->d.kind == ANTS_LRF_RZ && cfg->stat == ANTS_STAT_ML &&
                     set->d.na <= 64 && (G.nz == 3 || G.nz == 5 || G.nz == 7)) ||
                    ants::xf_applies(set->d, G);
  const int W[3] = {4, 2, 1}, B[2] = {0, 2};
  float best_ms = HUGE_VALF;
  int k = 0;
  hipError_t e = hipSuccess;
  for (int sc = 0; sc <= (fact ? 1 : 0) && e == hipSuccess; ++sc)
    for (int wi = 0; wi < 3 && e == hipSuccess; ++wi)
      for (int bi = 0; bi < 2 && e == hipSuccess; ++bi) {
        G.plan_screen = sc;
        G.plan_wpb = W[wi];
        G.plan_bpc = B[bi];
        e = ants::launch_grid(set->d, G, io, s, ants::num_cu() * 8);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(a, s);
        if (e == hipSuccess) e = ants::launch_grid(set->d, G, io, s, ants::num_cu() * 8);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) break;
        if (host_ms) host_ms[k] = ms;
        ++k;
        if (ms < best_ms) {
          best_ms = ms;
          *best = ants_grid_plan{W[wi], B[bi], sc};
        }
      }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return hip_fail(e, "ants_autotune");
  return ants_set_plan(set, cfg, best);
}

ants_status ants_generate(ants_lrfset* set, const ants_gen_cfg* cfg, int64_t n_events,
                          uint64_t seed, uint64_t first_event, float* d_signals, float* d_truth,
                          void* hip_stream) {
  if (!set || !cfg) return fail(ANTS_E_ARG, "ants_generate: NULL set or cfg");
  if (n_events < 0) return fail(ANTS_E_ARG, "n_events = %lld < 0", (long long)n_events);
  if (cfg->region != 0 && cfg->region != 1)
    return fail(ANTS_E_ARG, "region = %d must be 0 (disc) or 1 (square)", cfg->region);
  if (!(cfg->extent > 0.0 && isfinite(cfg->extent)))
    return fail(ANTS_E_ARG, "extent = %g must be positive", cfg->extent);
  if (!(cfg->e_lo >= 0.0 && cfg->e_hi >= cfg->e_lo && isfinite(cfg->e_hi)))
    return fail(ANTS_E_ARG, "energy range [%g, %g] invalid", cfg->e_lo, cfg->e_hi);
  if (!isfinite(cfg->z_lo) || !isfinite(cfg->z_hi))
    return fail(ANTS_E_ARG, "depth range not finite");
  if (n_events == 0) return ANTS_OK;
  if (!d_signals) return fail(ANTS_E_ARG, "d_signals is NULL");
  GenP P;
  memset(&P, 0, sizeof(P));
  P.n = n_events;
  P.first = first_event;
  P.k0 = (uint32_t)seed;
  P.k1 = (uint32_t)(seed >> 32);
  P.region = cfg->region;
  P.noiseless = cfg->noiseless ? 1 : 0;
  P.extent = cfg->extent;
  P.z_lo = cfg->z_lo;
  P.z_hi = cfg->z_hi;
  P.e_lo = cfg->e_lo;
  P.e_hi = cfg->e_hi;
  P.sig = d_signals;
  P.truth = d_truth;
  int dev = 0;
  hipGetDevice(&dev);
  if (dev != set->device)
    return fail(ANTS_E_ARG, "LRF set lives on device %d, current device is %d", set->device,
                dev);
  hipError_t e = ants::launch_gen(set->d, P, (hipStream_t)hip_stream, ants::num_cu() * 16);
  if (e != hipSuccess) return hip_fail(e, "ants_generate launch");
  return ANTS_OK;
}

}  // extern "C"
