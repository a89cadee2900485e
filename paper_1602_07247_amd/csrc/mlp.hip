// Learned seed for the contracting grid: a fully connected ReLU network
// (in the spirit of the artificial-neural-network reconstruction of
// Sec. 5.1.3, trained by back-propagation on events with known positions)
// mapping normalised sensor signals to a position seed and a log-variance.
//
// Storage: FP32 master weights, BF16 copies for the products; activations
// stored in BF16; every product accumulates in FP32 on the matrix cores
// (v_mfma_f32_16x16x32_bf16).
//
// GEMM convention: C[m][n] = sum_k A(m,k) * B(n,k), operands addressed with
// arbitrary element strides so the same kernel serves the forward product
// (A = activations, B = weights), the input gradient (B = weights seen
// transposed) and the weight gradient (A and B = batch-transposed views).
#include <math.h>

#include "ants_internal.h"

namespace ants {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, LDK = BK + 8;   // LDS row pitch (bf16 elements)

__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }   // round to nearest even

// Operand tile staging: a 64 x 32 tile X(r0 + i, k0 + j) into S[i][j] (LDS
// row pitch LDK), in two halves (global -> registers, registers -> LDS) so
// the next tile's loads are in flight during the current tile's products.
// Mode 0: k contiguous (X = base[r * s_r + k]), each thread loads 8
// consecutive k of one row; mode 1: rows contiguous (base[k * s_k + r], the
// batch-major operands of the weight gradients), each thread loads 8
// consecutive rows of one k and writes them down the tile's column; mode 2:
// any strides, element by element.  Elements past R or K are zero.
__device__ __forceinline__ bf16x8 load_tile(const __bf16* X, int64_t s_r, int64_t s_k, int R,
                                            int K, int r0, int k0, int mode, int tid) {
  bf16x8 v;
  if (mode == 1) {
    const int r = r0 + (tid & 7) * 8, k = k0 + (tid >> 3);
    if (k < K && r + 7 < R) {
      v = *(const bf16x8*)(X + (int64_t)k * s_k + r);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        v[e] = (k < K && r + e < R) ? X[(int64_t)k * s_k + r + e] : (__bf16)0.f;
    }
  } else {
    const int r = r0 + (tid >> 2), k = k0 + (tid & 3) * 8;
    if (mode == 0 && r < R && k + 7 < K) {
      v = *(const bf16x8*)(X + (int64_t)r * s_r + k);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e)
        v[e] = (r < R && k + e < K) ? X[(int64_t)r * s_r + (int64_t)(k + e) * s_k] : (__bf16)0.f;
    }
  }
  return v;
}
__device__ __forceinline__ void store_tile(bf16x8 v, int mode, __bf16* S, int tid) {
  if (mode == 1) {
    const int lk = tid >> 3, lr = (tid & 7) * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) S[(lr + e) * LDK + lk] = v[e];
  } else {
    *(bf16x8*)(S + (tid >> 2) * LDK + (tid & 3) * 8) = v;
  }
}

__device__ __forceinline__ void gemm_store(const GemmP& P, int m, int n, float v) {
  if (P.bias) v += P.bias[n];
  if (P.relu) v = fmaxf(v, 0.f);
  if (P.mask && !((float)P.mask[(int64_t)m * P.ldmask + n] > 0.f)) v = 0.f;
  if (P.Cf) P.Cf[(int64_t)m * P.ldcf + n] = v;
  if (P.Cb) P.Cb[(int64_t)m * P.ldcb + n] = to_bf16(v);
}

// Block (x, y, z): output tile (n0, m0) over the z-th of gridDim.z equal
// slices of k (whole BK steps).  One slice: the epilogue is applied here;
// several: the raw FP32 partial goes to ws[z][m][n] and gemm_reduce_kernel
// adds the slices in order (deterministic) and applies it.
__global__ void __launch_bounds__(256) gemm_kernel(GemmP P, int amode, int bmode, int kslice) {
  __shared__ __align__(16) __bf16 As[BM * LDK];
  __shared__ __align__(16) __bf16 Bs[BN * LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};

  const int kb = blockIdx.z * kslice;
  const int ke = kb + kslice < P.K ? kb + kslice : P.K;
  bf16x8 va, vb;
  if (kb < ke) {
    va = load_tile(P.A, P.sa_m, P.sa_k, P.M, ke, m0, kb, amode, tid);
    vb = load_tile(P.B, P.sb_n, P.sb_k, P.N, ke, n0, kb, bmode, tid);
  }
  for (int k0 = kb; k0 < ke; k0 += BK) {
    store_tile(va, amode, As, tid);
    store_tile(vb, bmode, Bs, tid);
    __syncthreads();
    if (k0 + BK < ke) {
      va = load_tile(P.A, P.sa_m, P.sa_k, P.M, ke, m0, k0 + BK, amode, tid);
      vb = load_tile(P.B, P.sb_n, P.sb_k, P.N, ke, n0, k0 + BK, bmode, tid);
    }
    // operand fragments: lane l holds row (l % 16) and k = 8*(l / 16) .. +7,
    // the same k assignment for A and B
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8*)(As + (wr + i * 16 + fr) * LDK + fk);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8*)(Bs + (wc + j * 16 + fr) * LDK + fk);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  // result layout: lane l holds C[4*(l/16) + r][l % 16], r = 0..3
  float* part = gridDim.z > 1 ? P.ws + (int64_t)blockIdx.z * P.M * P.N : nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wr + i * 16 + (lane >> 4) * 4 + r;
        const int n = n0 + wc + j * 16 + (lane & 15);
        if (m < P.M && n < P.N) {
          if (part) part[(int64_t)m * P.N + n] = acc[i][j][r];
          else gemm_store(P, m, n, acc[i][j][r]);
        }
      }
}

__global__ void gemm_reduce_kernel(GemmP P, int splits) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mn = (int64_t)P.M * P.N;
  if (i >= mn) return;
  // slices added in order; loads issued eight at a time
  float v = 0.f;
  int z = 0;
  for (; z + 8 <= splits; z += 8) {
    float t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = P.ws[(z + u) * mn + i];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += t[u];
  }
  for (; z < splits; ++z) v += P.ws[z * mn + i];
  gemm_store(P, (int)(i / P.N), (int)(i % P.N), v);
}

// ---------------------------------------------------------------------------
// Fused inference: one block of four waves runs FR events through every
// layer with the activations held in one LDS buffer (BF16, rows padded by
// 8 elements) that each layer overwrites in place: every wave first reads
// all of its operands into its accumulators, the block synchronises, then
// the outputs are written.  Weights are read from global memory
// (L2-resident) straight into the MFMA operand registers, one k-step ahead.  Each product is the
// same sequence of 16x16x32 MFMAs as in gemm_kernel (FP32 accumulators from
// zero, k ascending), so hidden activations and outputs equal that path's.
// Hidden width 256: wave w owns output columns 64w..64w+63 of every layer,
// for all FR events (RT row tiles of 16): each weight fragment read from L2
// feeds RT MFMAs.
constexpr int FR = 128, FH = 256, FPITCH = FH + 8, RT = FR / 16;

// kernel-argument arrays indexed with constants only (no private copies)
__device__ __forceinline__ const __bf16* fwd_w(const FwdP& P, int l) {
  return l == 0 ? P.W[0] : l == 1 ? P.W[1] : l == 2 ? P.W[2] : l == 3 ? P.W[3] : P.W[4];
}
__device__ __forceinline__ const float* fwd_b(const FwdP& P, int l) {
  return l == 0 ? P.b[0] : l == 1 ? P.b[1] : l == 2 ? P.b[2] : l == 3 ? P.b[3] : P.b[4];
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
mlp_fwd_kernel(FwdP P) {
  extern __shared__ __align__(16) __bf16 fsm[];
  __bf16* buf = fsm;                     // [FR][FPITCH] activations
  // before the first layer: FP32 signals in the first 16 KiB, the BF16
  // inputs [FR][kin + 8] after them
  __bf16* inb = fsm + FR * 64 * 2;
  __shared__ float scl[FR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t e0 = (int64_t)blockIdx.x * FR;
  const int fr = lane & 15, fk = (lane >> 4) * 8;

  // inputs x = bf16(n_a * (n_active / N)), as normalize_kernel: the block's
  // signals are first staged in LDS by all threads (independent loads),
  // then each event's sum runs in sensor order as there
  float* stage = (float*)buf;            // [FR][na] FP32, na <= 64
  const int na = P.na;
  for (int i = tid; i < FR * na; i += 256) {
    const int r = i / na, a = i - r * na;
    const int64_t e = e0 + r;
    stage[i] = e < P.n ? P.sig[e * P.ld + P.col[a]] : 0.f;
  }
  __syncthreads();
  if (tid < FR) {
    const int64_t e = e0 + tid;
    float sc = 0.f;
    if (e < P.n) {
      const float* row = stage + tid * na;
      float N = 0.f;
      bool ok = true;
      for (int a = 0; a < na; ++a) {
        const float v = row[a];
        if (!(v >= 0.f) || !(v < __builtin_huge_valf())) ok = false;
        N += v;
      }
      ok = ok && N > 0.f;
      sc = ok ? (float)na / N : 0.f;
    }
    scl[tid] = sc;
  }
  __syncthreads();
  const int kin = P.kin, pin = kin + 8;
  for (int i = tid; i < FR * kin; i += 256) {
    const int r = i / kin, a = i - r * kin;
    __bf16 v = (__bf16)0.f;
    if (a < na && scl[r] > 0.f) v = to_bf16(stage[r * na + a] * scl[r]);
    inb[r * pin + a] = v;
  }
  __syncthreads();

  const __bf16* in = inb;
  int pitch = pin, din = kin;
#pragma unroll
  for (int l = 0; l < kFwdMaxLayers; ++l) {
    if (l >= P.layers) break;
    const __bf16* W = fwd_w(P, l);
    f32x4 acc[RT][4];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    bf16x8 b[4], bn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *(const bf16x8*)(W + (int64_t)(wave * 64 + j * 16 + fr) * din + fk);
    for (int k0 = 0; k0 < din; k0 += 32) {
      if (k0 + 32 < din) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          bn[j] = *(const bf16x8*)(W + (int64_t)(wave * 64 + j * 16 + fr) * din + k0 + 32 + fk);
      }
      bf16x8 a[RT];
#pragma unroll
      for (int i = 0; i < RT; ++i) a[i] = *(const bf16x8*)(in + (i * 16 + fr) * pitch + k0 + fk);
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = bn[j];
    }
    // every wave has read its operands: bias, ReLU, BF16 in place
    __syncthreads();
    const float* bias = fwd_b(P, l);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = wave * 64 + j * 16 + fr;
      const float bc = bias[c];
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          buf[(i * 16 + (lane >> 4) * 4 + r) * FPITCH + c] = to_bf16(fmaxf(acc[i][j][r] + bc, 0.f));
    }
    __syncthreads();
    in = buf;
    pitch = FPITCH;
    din = FH;
  }

  // output layer (4 rows of weights, padded to one 16-column tile): wave w
  // takes the row tiles w, w + 4, ... (events 16 t..16 t + 15 of tile t)
  {
    const __bf16* W = fwd_w(P, P.layers);
#pragma unroll
    for (int u = 0; u < RT / 4; ++u) {
      const int t = wave + 4 * u;
      f32x4 acc = (f32x4){0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < FH; k0 += 32) {
        bf16x8 bb;
        if (fr < 4) {
          bb = *(const bf16x8*)(W + (int64_t)fr * FH + k0 + fk);
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) bb[q] = (__bf16)0.f;
        }
        const bf16x8 a = *(const bf16x8*)(in + (t * 16 + fr) * FPITCH + k0 + fk);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bb, acc, 0, 0, 0);
      }
      if (fr < 4) {
        const float bc = fwd_b(P, P.layers)[fr];
        const float sc = fr == 0 ? P.scale[0] : fr == 1 ? P.scale[1] : P.scale[2];
        const float of = fr == 0 ? P.offset[0] : fr == 1 ? P.offset[1] : P.offset[2];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t e = e0 + t * 16 + (lane >> 4) * 4 + r;
          if (e < P.n) {
            const float y = acc[r] + bc;
            P.out[e * 4 + fr] = (P.seeds && fr < 3) ? of + sc * y : y;
          }
        }
      }
    }
  }
}

// x_hat = bf16(n_a * (n_active / N)) for the active sensors, zero padding.
// A block takes 64 events: their signals are staged in LDS by all threads,
// each event's sum runs in sensor order (as in the fused inference), and
// the rows are written by all threads.
constexpr int NR = 64;
__global__ void __launch_bounds__(256) normalize_kernel(const float* sig, int64_t ld,
                                                        const int32_t* col, int na, int64_t n,
                                                        int kin, __bf16* X) {
  __shared__ float stage[NR * 64];
  __shared__ float scl[NR];
  const int tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * NR;
  for (int i = tid; i < NR * na; i += 256) {
    const int r = i / na, a = i - r * na;
    const int64_t e = e0 + r;
    stage[i] = e < n ? sig[e * ld + col[a]] : 0.f;
  }
  __syncthreads();
  if (tid < NR) {
    const float* row = stage + tid * na;
    float N = 0.f;
    bool ok = e0 + tid < n;
    for (int a = 0; a < na; ++a) {
      const float v = row[a];
      if (!(v >= 0.f) || !(v < __builtin_huge_valf())) ok = false;
      N += v;
    }
    ok = ok && N > 0.f;
    scl[tid] = ok ? (float)na / N : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < NR * kin; i += 256) {
    const int r = i / kin, a = i - r * kin;
    const int64_t e = e0 + r;
    if (e >= n) continue;
    __bf16 v = (__bf16)0.f;
    if (a < na && scl[r] > 0.f) v = to_bf16(stage[r * na + a] * scl[r]);
    X[e * kin + a] = v;
  }
}

// Gaussian negative log-likelihood with one log-variance s per event:
//   loss = 0.5 exp(-s) |p - t|^2 + 1.5 s, targets t = (pos - offset) / scale.
// Writes dY = dloss/dY / batch (FP32 and BF16) and the per-event loss.
__global__ void head_loss_kernel(const float* Y, const float* target, int64_t ldt, int64_t n,
                                 HeadP H, float* dY, __bf16* dYb, float* loss) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float* y = Y + e * 4;
  float r2 = 0.f, r[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float t = (target[e * ldt + c] - H.offset[c]) * H.inv_scale[c];
    r[c] = y[c] - t;
    r2 = fmaf(r[c], r[c], r2);
  }
  const float s = y[3], es = expf(-s), w = H.inv_batch;
  float g[4] = {es * r[0] * w, es * r[1] * w, es * r[2] * w, (1.5f - 0.5f * es * r2) * w};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    dY[e * 4 + c] = g[c];
    dYb[e * 4 + c] = to_bf16(g[c]);
  }
  loss[e] = 0.5f * es * r2 + 1.5f * s;
}

// dH3 = (dY W4) * [H3 > 0], FP32 sums of four products, stored in BF16
__global__ void head_back_kernel(const float* dY, const float* W4, const __bf16* H3, int64_t n,
                                 int hidden, __bf16* dH) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * hidden) return;
  const int64_t e = i / hidden;
  const int j = (int)(i - e * hidden);
  float v = 0.f;
#pragma unroll
  for (int o = 0; o < 4; ++o) v = fmaf(dY[e * 4 + o], (float)(__bf16)W4[o * hidden + j], v);
  dH[i] = ((float)H3[i] > 0.f) ? to_bf16(v) : (__bf16)0.f;
}

// column sums (bias gradients), deterministic: one block per column
__global__ void __launch_bounds__(256) colsum_bf16_kernel(const __bf16* D, int64_t n, int ld,
                                                          float* out) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int64_t e = threadIdx.x; e < n; e += 256) s += (float)D[e * ld + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}
__global__ void __launch_bounds__(256) colsum_f32_kernel(const float* D, int64_t n, int ld,
                                                         float* out) {
  __shared__ float red[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (int64_t e = threadIdx.x; e < n; e += 256) s += D[e * ld + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

__global__ void sum_f32_kernel(const float* v, int64_t n, float scale, float* out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int64_t e = threadIdx.x; e < n; e += 256) s += v[e];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] * scale;
}

// Adam (Kingma and Ba) on the FP32 master copy; refreshes the BF16 copy
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, __bf16* pb, int64_t n,
                            AdamP A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = A.b1 * m[i] + (1.f - A.b1) * gi;
  const float vi = A.b2 * v[i] + (1.f - A.b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float upd = A.lr * (mi * A.c1) / (sqrtf(vi * A.c2) + A.eps);
  const float pn = p[i] - upd;
  p[i] = pn;
  pb[i] = to_bf16(pn);
}

__global__ void to_bf16_kernel(const float* p, __bf16* pb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pb[i] = to_bf16(p[i]);
}

// network output (normalised) -> seed in mm: pos = offset + scale * y, s kept

inline unsigned nb(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// staging mode of an operand (see stage_tile): vector loads need 16-byte
// aligned rows (or columns) and a unit stride along the loaded direction
static int stage_mode(const __bf16* X, int64_t s_r, int64_t s_k) {
  const bool al = ((uintptr_t)X & 15) == 0;
  if (al && s_k == 1 && s_r % 8 == 0) return 0;
  if (al && s_r == 1 && s_k % 8 == 0) return 1;
  return 2;
}

hipError_t launch_gemm(const GemmP& P, hipStream_t s) {
  if (P.M <= 0 || P.N <= 0) return hipSuccess;
  int splits = P.ws ? gemm_splits(P.M, P.N, P.K) : 1;
  if ((int64_t)splits * P.M * P.N > P.ws_n) splits = 1;
  // whole BK steps per slice
  const int steps = P.K > 0 ? (P.K + BK - 1) / BK : 0;
  const int per = steps > 0 ? (steps + splits - 1) / splits : 1;
  splits = steps > 0 ? (steps + per - 1) / per : 1;
  const int kslice = per * BK;
  dim3 g((unsigned)((P.N + BN - 1) / BN), (unsigned)((P.M + BM - 1) / BM), (unsigned)splits);
  hipLaunchKernelGGL(gemm_kernel, g, dim3(256), 0, s, P, stage_mode(P.A, P.sa_m, P.sa_k),
                     stage_mode(P.B, P.sb_n, P.sb_k), kslice);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && splits > 1) {
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3(nb((int64_t)P.M * P.N)), dim3(256), 0, s, P,
                       splits);
    e = hipGetLastError();
  }
  return e;
}
hipError_t launch_mlp_fwd(const FwdP& P, hipStream_t s) {
  if (P.n <= 0) return hipSuccess;
  if (P.kin > FH || P.kin % 32 || P.layers < 1 || P.layers > kFwdMaxLayers || P.na > 64 ||
      P.na > P.kin)
    return hipErrorInvalidValue;
  // the activations, or before the first layer the FP32 signal stage
  // [FR][64] followed by the BF16 inputs [FR][kin + 8], whichever is larger
  const size_t act = (size_t)FR * FPITCH * sizeof(__bf16);
  const size_t pre = (size_t)FR * 64 * sizeof(float) + (size_t)FR * (P.kin + 8) * sizeof(__bf16);
  const size_t smem = act > pre ? act : pre;
  hipError_t e = hipFuncSetAttribute((const void*)mlp_fwd_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_fwd_kernel, dim3((unsigned)((P.n + FR - 1) / FR)), dim3(256), smem, s, P);
  return hipGetLastError();
}
hipError_t launch_normalize(const float* sig, int64_t ld, const int32_t* col, int na, int64_t n,
                            int kin, __bf16* X, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (na > 64 || na > kin) return hipErrorInvalidValue;
  hipLaunchKernelGGL(normalize_kernel, dim3(nb(n, NR)), dim3(256), 0, s, sig, ld, col, na, n, kin,
                     X);
  return hipGetLastError();
}
hipError_t launch_head_loss(const float* Y, const float* target, int64_t ldt, int64_t n,
                            const HeadP& H, float* dY, __bf16* dYb, float* loss, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(head_loss_kernel, dim3(nb(n)), dim3(256), 0, s, Y, target, ldt, n, H, dY,
                     dYb, loss);
  return hipGetLastError();
}
hipError_t launch_head_back(const float* dY, const float* W4, const __bf16* H3, int64_t n,
                            int hidden, __bf16* dH, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(head_back_kernel, dim3(nb(n * hidden)), dim3(256), 0, s, dY, W4, H3, n,
                     hidden, dH);
  return hipGetLastError();
}
hipError_t launch_colsum_bf16(const __bf16* D, int64_t n, int ld, int cols, float* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(colsum_bf16_kernel, dim3(cols), dim3(256), 0, s, D, n, ld, out);
  return hipGetLastError();
}
hipError_t launch_colsum_f32(const float* D, int64_t n, int ld, int cols, float* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(colsum_f32_kernel, dim3(cols), dim3(256), 0, s, D, n, ld, out);
  return hipGetLastError();
}
hipError_t launch_sum_f32(const float* v, int64_t n, float scale, float* out, hipStream_t s) {
  hipLaunchKernelGGL(sum_f32_kernel, dim3(1), dim3(256), 0, s, v, n, scale, out);
  return hipGetLastError();
}
hipError_t launch_adam(float* p, const float* g, float* m, float* v, __bf16* pb, int64_t n,
                       const AdamP& A, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3(nb(n)), dim3(256), 0, s, p, g, m, v, pb, n, A);
  return hipGetLastError();
}
hipError_t launch_to_bf16(const float* p, __bf16* pb, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, dim3(nb(n)), dim3(256), 0, s, p, pb, n);
  return hipGetLastError();
}

}  // namespace ants
