// Host side of the learned seed (network handle, forward, gradient, Adam
// training) and of the seeded reconstruction (network -> seeds ->
// refinement grid -> chi2/ndf fallback to the full grid).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "ants_internal.h"

using namespace ants;

namespace {

constexpr int kMaxBatch = 65536;

struct Dev {
  std::vector<void*> bufs;
  template <class T>
  hipError_t alloc(T** p, size_t n) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T) + 16);
    if (e == hipSuccess) bufs.push_back(*p);
    return e;
  }
  ~Dev() {
    for (void* b : bufs) (void)hipFree(b);
  }
};

}  // namespace

struct ants_mlp {
  ants_mlp_cfg cfg;
  int nin_pad, hidden, layers;
  int64_t nparams;
  std::vector<int64_t> offW, offB, din, dout;   // layers + 1 (last = head)
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *best = nullptr;
  __bf16* pb = nullptr;
  int64_t t = 0;
  int device = 0;
  HeadP head;
  // activations for up to `rows` events
  int64_t rows = 0;
  __bf16* X = nullptr;
  std::vector<__bf16*> H;
  float *Y = nullptr, *dY = nullptr, *loss_ev = nullptr, *loss = nullptr;
  __bf16 *dYb = nullptr, *dHa = nullptr, *dHb = nullptr;
  float* gws = nullptr;   // split-K partial products of the weight gradients
  int64_t gws_n = 0;
  Dev mem;      // parameter-sized buffers
  Dev work;     // activation buffers (reallocated when rows grow)
};

namespace {

ants_status mlp_workspace(ants_mlp* M, int64_t rows) {
  if (M->rows >= rows) return ANTS_OK;
  for (void* b : M->work.bufs) (void)hipFree(b);
  M->work.bufs.clear();
  M->H.assign(M->layers, nullptr);
  hipError_t e = M->work.alloc(&M->X, (size_t)rows * M->nin_pad);
  for (int l = 0; l < M->layers && e == hipSuccess; ++l)
    e = M->work.alloc(&M->H[l], (size_t)rows * M->hidden);
  if (e == hipSuccess) e = M->work.alloc(&M->Y, (size_t)rows * 4);
  if (e == hipSuccess) e = M->work.alloc(&M->dY, (size_t)rows * 4);
  if (e == hipSuccess) e = M->work.alloc(&M->dYb, (size_t)rows * 4);
  if (e == hipSuccess) e = M->work.alloc(&M->dHa, (size_t)rows * M->hidden);
  if (e == hipSuccess) e = M->work.alloc(&M->dHb, (size_t)rows * M->hidden);
  if (e == hipSuccess) e = M->work.alloc(&M->loss_ev, (size_t)rows);
  if (e == hipSuccess) e = M->work.alloc(&M->loss, 4);
  // the weight gradients' split-K partials at this many rows (the split
  // only grows with the row count)
  int64_t ws = (int64_t)gemm_splits(4, M->hidden, (int)rows) * 4 * M->hidden;
  for (int l = 0; l < M->layers; ++l) {
    const int64_t w = (int64_t)gemm_splits(M->hidden, (int)M->din[l], (int)rows) * M->hidden *
                      M->din[l];
    ws = w > ws ? w : ws;
  }
  M->gws_n = ws;
  if (e == hipSuccess) e = M->work.alloc(&M->gws, (size_t)ws);
  if (e != hipSuccess) {
    M->rows = 0;
    return hip_error(e, "network workspace");
  }
  M->rows = rows;
  return ANTS_OK;
}

GemmP gemm(int Mr, int N, int K, const __bf16* A, int64_t sam, int64_t sak, const __bf16* B,
           int64_t sbn, int64_t sbk) {
  GemmP P;
  memset(&P, 0, sizeof(P));
  P.M = Mr;
  P.N = N;
  P.K = K;
  P.A = A;
  P.sa_m = sam;
  P.sa_k = sak;
  P.B = B;
  P.sb_n = sbn;
  P.sb_k = sbk;
  return P;
}

// forward of `n` rows (n <= M->rows): X -> H[0..L-1] -> Y
hipError_t forward_rows(ants_mlp* M, const ants_lrfset* S, const float* sig, int64_t n,
                        hipStream_t s) {
  hipError_t e = launch_normalize(sig, S->ns, S->d.col, S->d.na, n, M->nin_pad, M->X, s);
  const __bf16* in = M->X;
  for (int l = 0; l < M->layers && e == hipSuccess; ++l) {
    GemmP P = gemm((int)n, M->hidden, (int)M->din[l], in, M->din[l], 1, M->pb + M->offW[l],
                   M->din[l], 1);
    P.bias = M->p + M->offB[l];
    P.relu = 1;
    P.Cb = M->H[l];
    P.ldcb = M->hidden;
    e = launch_gemm(P, s);
    in = M->H[l];
  }
  if (e == hipSuccess) {
    const int L = M->layers;
    GemmP P = gemm((int)n, 4, M->hidden, in, M->hidden, 1, M->pb + M->offW[L], M->hidden, 1);
    P.bias = M->p + M->offB[L];
    P.Cf = M->Y;
    P.ldcf = 4;
    e = launch_gemm(P, s);
  }
  return e;
}

// Fused inference over n events (no workspace): raw outputs or seeds.
hipError_t infer(const ants_mlp* M, const ants_lrfset* S, const float* sig, int64_t n, float* out,
                 bool seeds, hipStream_t s) {
  FwdP P;
  memset(&P, 0, sizeof(P));
  P.sig = sig;
  P.ld = S->ns;
  P.col = S->d.col;
  P.na = S->d.na;
  P.n = n;
  P.kin = M->nin_pad;
  P.layers = M->layers;
  for (int l = 0; l <= M->layers; ++l) {
    P.W[l] = M->pb + M->offW[l];
    P.b[l] = M->p + M->offB[l];
  }
  P.out = out;
  P.seeds = seeds ? 1 : 0;
  for (int a = 0; a < 3; ++a) {
    P.scale[a] = M->head.scale[a];
    P.offset[a] = M->head.offset[a];
  }
  return launch_mlp_fwd(P, s);
}

// loss and gradient of the mean loss over n rows (forward must have run)
hipError_t backward_rows(ants_mlp* M, const float* target, int64_t ldt, int64_t n, hipStream_t s) {
  HeadP H = M->head;
  H.inv_batch = 1.0f / (float)n;
  hipError_t e = launch_head_loss(M->Y, target, ldt, n, H, M->dY, M->dYb, M->loss_ev, s);
  const int L = M->layers;
  if (e == hipSuccess) e = launch_colsum_f32(M->dY, n, 4, 4, M->g + M->offB[L], s);
  if (e == hipSuccess) {
    // dW_out[o][j] = sum_b dY[b][o] H[L-1][b][j]
    GemmP P = gemm(4, M->hidden, (int)n, M->dYb, 1, 4, M->H[L - 1], 1, M->hidden);
    P.ws = M->gws;
    P.ws_n = M->gws_n;
    P.Cf = M->g + M->offW[L];
    P.ldcf = M->hidden;
    e = launch_gemm(P, s);
  }
  if (e == hipSuccess)
    e = launch_head_back(M->dY, M->p + M->offW[L], M->H[L - 1], n, M->hidden, M->dHa, s);
  __bf16* dH = M->dHa;
  __bf16* dHn = M->dHb;
  for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
    e = launch_colsum_bf16(dH, n, M->hidden, M->hidden, M->g + M->offB[l], s);
    const __bf16* in = l == 0 ? M->X : M->H[l - 1];
    const int64_t di = M->din[l];
    if (e == hipSuccess) {
      // dW_l[j][i] = sum_b dH[b][j] in[b][i]
      GemmP P = gemm(M->hidden, (int)di, (int)n, dH, 1, M->hidden, in, 1, di);
      P.ws = M->gws;
      P.ws_n = M->gws_n;
      P.Cf = M->g + M->offW[l];
      P.ldcf = di;
      e = launch_gemm(P, s);
    }
    if (l > 0 && e == hipSuccess) {
      // dH_prev[b][i] = sum_j dH[b][j] W_l[j][i], times ReLU'(H[l-1])
      GemmP P = gemm((int)n, (int)di, M->hidden, dH, M->hidden, 1, M->pb + M->offW[l], 1, di);
      P.mask = M->H[l - 1];
      P.ldmask = M->hidden;
      P.Cb = dHn;
      P.ldcb = di;
      e = launch_gemm(P, s);
      __bf16* t = dH;
      dH = dHn;
      dHn = t;
    }
  }
  if (e == hipSuccess) e = launch_sum_f32(M->loss_ev, n, 1.0f / (float)n, M->loss, s);
  return e;
}

ants_status check_pair(const ants_mlp* M, const ants_lrfset* S) {
  if (!M || !S) return set_error(ANTS_E_ARG, "NULL network or LRF set");
  if (S->d.na != M->cfg.n_in)
    return set_error(ANTS_E_ARG, "network has %d inputs but the LRF set has %d active sensors",
                     M->cfg.n_in, S->d.na);
  int dev = 0;
  hipGetDevice(&dev);
  if (dev != M->device || dev != S->device)
    return set_error(ANTS_E_ARG, "network, LRF set and current device differ");
  return ANTS_OK;
}

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

hipError_t adam_step(ants_mlp* M, const ants_adam_cfg* A, hipStream_t s) {
  M->t += 1;
  AdamP P;
  P.lr = (float)A->lr;
  P.b1 = (float)A->beta1;
  P.b2 = (float)A->beta2;
  P.eps = (float)A->eps;
  P.c1 = (float)(1.0 / (1.0 - pow(A->beta1, (double)M->t)));
  P.c2 = (float)(1.0 / (1.0 - pow(A->beta2, (double)M->t)));
  return launch_adam(M->p, M->g, M->m, M->v, M->pb, M->nparams, P, s);
}

ants_status check_adam(const ants_adam_cfg* A) {
  if (!A) return set_error(ANTS_E_ARG, "NULL Adam configuration");
  if (!(A->lr > 0.0 && A->beta1 >= 0.0 && A->beta1 < 1.0 && A->beta2 >= 0.0 && A->beta2 < 1.0 &&
        A->eps > 0.0))
    return set_error(ANTS_E_ARG, "Adam: need lr > 0, 0 <= beta < 1, eps > 0");
  return ANTS_OK;
}

}  // namespace

extern "C" {

ants_status ants_mlp_create(const ants_mlp_cfg* cfg, ants_mlp** out) {
  if (!out) return set_error(ANTS_E_ARG, "ants_mlp_create: NULL out");
  *out = nullptr;
  if (!cfg) return set_error(ANTS_E_ARG, "ants_mlp_create: NULL cfg");
  if (cfg->n_in < 1 || cfg->n_in > 64)
    return set_error(ANTS_E_ARG, "n_in = %d outside 1..64", cfg->n_in);
  if (cfg->hidden != 256)
    return set_error(ANTS_E_UNSUPPORTED, "hidden = %d (only 256 is built)", cfg->hidden);
  if (cfg->n_layers < 1 || cfg->n_layers > 4)
    return set_error(ANTS_E_ARG, "n_layers = %d outside 1..4", cfg->n_layers);
  for (int a = 0; a < 3; ++a)
    if (!(cfg->pos_scale[a] > 0.0 && isfinite(cfg->pos_scale[a]) && isfinite(cfg->pos_offset[a])))
      return set_error(ANTS_E_ARG, "pos_scale must be positive and offsets finite");
  ants_mlp* M = new ants_mlp();
  M->cfg = *cfg;
  M->nin_pad = (cfg->n_in + 31) / 32 * 32;
  M->hidden = cfg->hidden;
  M->layers = cfg->n_layers;
  hipGetDevice(&M->device);
  int64_t off = 0;
  for (int l = 0; l <= M->layers; ++l) {
    int64_t di = l == 0 ? M->nin_pad : M->hidden;
    int64_t dout = l == M->layers ? 4 : M->hidden;
    M->din.push_back(di);
    M->dout.push_back(dout);
    M->offW.push_back(off);
    off += di * dout;
    M->offB.push_back(off);
    off += dout;
  }
  M->nparams = off;
  for (int c = 0; c < 3; ++c) {
    M->head.scale[c] = (float)cfg->pos_scale[c];
    M->head.inv_scale[c] = (float)(1.0 / cfg->pos_scale[c]);
    M->head.offset[c] = (float)cfg->pos_offset[c];
  }
  M->head.inv_batch = 1.f;
  // He-uniform initialisation on the host: w ~ U(-b, b), b = sqrt(6 / fan_in);
  // padded input columns and biases are zero
  std::vector<float> h((size_t)M->nparams, 0.f);
  uint64_t st = cfg->seed;
  for (int l = 0; l <= M->layers; ++l) {
    int fan = l == 0 ? cfg->n_in : M->hidden;
    double b = sqrt(6.0 / fan);
    for (int64_t o = 0; o < M->dout[l]; ++o)
      for (int64_t i = 0; i < M->din[l]; ++i) {
        double u = (double)(splitmix64(st) >> 11) * 0x1.0p-53;
        float w = (l == 0 && i >= cfg->n_in) ? 0.f : (float)((2.0 * u - 1.0) * b);
        h[(size_t)(M->offW[l] + o * M->din[l] + i)] = w;
      }
  }
  hipError_t e = M->mem.alloc(&M->p, (size_t)M->nparams);
  if (e == hipSuccess) e = M->mem.alloc(&M->g, (size_t)M->nparams);
  if (e == hipSuccess) e = M->mem.alloc(&M->m, (size_t)M->nparams);
  if (e == hipSuccess) e = M->mem.alloc(&M->v, (size_t)M->nparams);
  if (e == hipSuccess) e = M->mem.alloc(&M->best, (size_t)M->nparams);
  if (e == hipSuccess) e = M->mem.alloc(&M->pb, (size_t)M->nparams);
  if (e != hipSuccess) {
    delete M;
    return hip_error(e, "ants_mlp_create");
  }
  ants_status stt = ants_mlp_set_params(M, h.data(), M->nparams);
  if (stt != ANTS_OK) {
    delete M;
    return stt;
  }
  *out = M;
  return ANTS_OK;
}

ants_status ants_mlp_destroy(ants_mlp* M) {
  delete M;
  return ANTS_OK;
}

int64_t ants_mlp_num_params(const ants_mlp* M) { return M ? M->nparams : 0; }

ants_status ants_mlp_get_params(const ants_mlp* M, float* host, int64_t n) {
  if (!M || !host) return set_error(ANTS_E_ARG, "ants_mlp_get_params: NULL argument");
  if (n != M->nparams) return set_error(ANTS_E_ARG, "n = %lld, network has %lld parameters",
                                        (long long)n, (long long)M->nparams);
  hipError_t e = hipMemcpy(host, M->p, n * sizeof(float), hipMemcpyDeviceToHost);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_mlp_get_params");
}

ants_status ants_mlp_set_params(ants_mlp* M, const float* host, int64_t n) {
  if (!M || !host) return set_error(ANTS_E_ARG, "ants_mlp_set_params: NULL argument");
  if (n != M->nparams) return set_error(ANTS_E_ARG, "n = %lld, network has %lld parameters",
                                        (long long)n, (long long)M->nparams);
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(host[i])) return set_error(ANTS_E_FORMAT, "parameter %lld not finite",
                                             (long long)i);
  hipError_t e = hipMemcpy(M->p, host, n * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(M->m, 0, n * sizeof(float));
  if (e == hipSuccess) e = hipMemset(M->v, 0, n * sizeof(float));
  if (e == hipSuccess) e = hipMemset(M->g, 0, n * sizeof(float));
  if (e == hipSuccess) e = launch_to_bf16(M->p, M->pb, n, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  M->t = 0;
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_mlp_set_params");
}

ants_status ants_mlp_forward(ants_mlp* M, const ants_lrfset* S, int64_t n, const float* d_signals,
                             float* d_pred, void* hip_stream) {
  ants_status st = check_pair(M, S);
  if (st != ANTS_OK) return st;
  if (n < 0) return set_error(ANTS_E_ARG, "n < 0");
  if (n == 0) return ANTS_OK;
  if (!d_signals || !d_pred) return set_error(ANTS_E_ARG, "NULL device pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = infer(M, S, d_signals, n, d_pred, false, s);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_mlp_forward");
}

ants_status ants_mlp_grad(ants_mlp* M, const ants_lrfset* S, int64_t n, const float* d_signals,
                          const float* d_target, float* d_grad, float* d_loss, void* hip_stream) {
  ants_status st = check_pair(M, S);
  if (st != ANTS_OK) return st;
  if (n < 1 || n > kMaxBatch) return set_error(ANTS_E_ARG, "batch n = %lld outside 1..%d",
                                               (long long)n, kMaxBatch);
  if (!d_signals || !d_target || !d_grad || !d_loss)
    return set_error(ANTS_E_ARG, "NULL device pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  st = mlp_workspace(M, n);
  if (st != ANTS_OK) return st;
  hipError_t e = forward_rows(M, S, d_signals, n, s);
  if (e == hipSuccess) e = backward_rows(M, d_target, 3, n, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d_grad, M->g, M->nparams * sizeof(float), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_loss, M->loss, sizeof(float), hipMemcpyDeviceToDevice, s);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_mlp_grad");
}

ants_status ants_mlp_train_step(ants_mlp* M, const ants_lrfset* S, int64_t n,
                                const float* d_signals, const float* d_target,
                                const ants_adam_cfg* adam, float* d_loss, void* hip_stream) {
  ants_status st = check_pair(M, S);
  if (st != ANTS_OK) return st;
  st = check_adam(adam);
  if (st != ANTS_OK) return st;
  if (n < 1 || n > kMaxBatch) return set_error(ANTS_E_ARG, "batch n = %lld outside 1..%d",
                                               (long long)n, kMaxBatch);
  if (!d_signals || !d_target) return set_error(ANTS_E_ARG, "NULL device pointer");
  hipStream_t s = (hipStream_t)hip_stream;
  st = mlp_workspace(M, n);
  if (st != ANTS_OK) return st;
  hipError_t e = forward_rows(M, S, d_signals, n, s);
  if (e == hipSuccess) e = backward_rows(M, d_target, 3, n, s);
  if (e == hipSuccess) e = adam_step(M, adam, s);
  if (e == hipSuccess && d_loss)
    e = hipMemcpyAsync(d_loss, M->loss, sizeof(float), hipMemcpyDeviceToDevice, s);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_mlp_train_step");
}

ants_status ants_mlp_train(ants_mlp* M, const ants_lrfset* Sc, const ants_train_cfg* C,
                           double* host_losses, void* hip_stream) {
  ants_lrfset* S = const_cast<ants_lrfset*>(Sc);
  ants_status st = check_pair(M, S);
  if (st != ANTS_OK) return st;
  if (!C) return set_error(ANTS_E_ARG, "NULL training configuration");
  st = check_adam(&C->adam);
  if (st != ANTS_OK) return st;
  if (C->batch < 1 || C->batch > kMaxBatch || C->n_train < C->batch || C->n_val < 1 ||
      C->epochs < 1 || !(C->lr_decay > 0.0 && C->lr_decay <= 1.0))
    return set_error(ANTS_E_ARG, "training sizes invalid (batch 1..%d <= n_train, n_val >= 1, "
                                 "epochs >= 1, 0 < lr_decay <= 1)", kMaxBatch);
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t ntot = C->n_train + C->n_val;
  Dev data;
  float *sig = nullptr, *truth = nullptr, *vloss = nullptr;
  hipError_t e = data.alloc(&sig, (size_t)ntot * S->ns);
  if (e == hipSuccess) e = data.alloc(&truth, (size_t)ntot * 4);
  if (e == hipSuccess) e = data.alloc(&vloss, 2);
  if (e != hipSuccess) return hip_error(e, "training data");
  st = ants_generate(S, &C->events, ntot, C->seed, 0, sig, truth, hip_stream);
  if (st != ANTS_OK) return st;
  const int64_t vchunk = C->n_val < kMaxBatch ? C->n_val : kMaxBatch;
  st = mlp_workspace(M, (int64_t)C->batch > vchunk ? (int64_t)C->batch : vchunk);
  if (st != ANTS_OK) return st;
  ants_adam_cfg A = C->adam;
  const int64_t steps = C->n_train / C->batch;
  double best = HUGE_VAL;
  std::vector<float> lbuf(2);
  for (int ep = 0; ep < C->epochs; ++ep) {
    double tr = 0.0;
    std::vector<float> hl((size_t)steps);
    for (int64_t b = 0; b < steps && e == hipSuccess; ++b) {
      e = forward_rows(M, S, sig + b * C->batch * S->ns, C->batch, s);
      if (e == hipSuccess) e = backward_rows(M, truth + b * C->batch * 4, 4, C->batch, s);
      if (e == hipSuccess) e = adam_step(M, &A, s);
      if (e == hipSuccess && (b % 64 == 0 || b == steps - 1)) {
        float lv = 0.f;
        e = hipMemcpyAsync(&lv, M->loss, sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        tr = lv;   // last sampled batch loss
      }
    }
    // validation loss (no update)
    double vsum = 0.0;
    for (int64_t b = 0; b < C->n_val && e == hipSuccess; b += vchunk) {
      int64_t r = C->n_val - b < vchunk ? C->n_val - b : vchunk;
      const int64_t row = C->n_train + b;
      e = forward_rows(M, S, sig + row * S->ns, r, s);
      HeadP H = M->head;
      H.inv_batch = 1.f;
      if (e == hipSuccess)
        e = launch_head_loss(M->Y, truth + row * 4, 4, r, H, M->dY, M->dYb, M->loss_ev, s);
      if (e == hipSuccess) e = launch_sum_f32(M->loss_ev, r, 1.0f, vloss, s);
      float lv = 0.f;
      if (e == hipSuccess) e = hipMemcpyAsync(&lv, vloss, sizeof(float), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      vsum += lv;
    }
    if (e != hipSuccess) return hip_error(e, "ants_mlp_train");
    const double val = vsum / (double)C->n_val;
    if (host_losses) {
      host_losses[2 * ep] = tr;
      host_losses[2 * ep + 1] = val;
    }
    if (val < best) {
      best = val;
      e = hipMemcpyAsync(M->best, M->p, M->nparams * sizeof(float), hipMemcpyDeviceToDevice, s);
    }
    A.lr *= C->lr_decay;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(M->p, M->best, M->nparams * sizeof(float), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = launch_to_bf16(M->p, M->pb, M->nparams, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_mlp_train");
}

ants_status ants_mlp_save(const ants_mlp* M, const char* path) {
  if (!M || !path) return set_error(ANTS_E_ARG, "ants_mlp_save: NULL argument");
  std::vector<float> h((size_t)M->nparams);
  ants_status st = ants_mlp_get_params(M, h.data(), M->nparams);
  if (st != ANTS_OK) return st;
  FILE* f = fopen(path, "wb");
  if (!f) return set_error(ANTS_E_ARG, "cannot open %s for writing", path);
  bool ok = fwrite("ANTSMLP1", 1, 8, f) == 8 && fwrite(&M->cfg, sizeof(M->cfg), 1, f) == 1 &&
            fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? ANTS_OK : set_error(ANTS_E_DEVICE, "write to %s failed", path);
}

ants_status ants_mlp_load(const char* path, ants_mlp** out) {
  if (!path || !out) return set_error(ANTS_E_ARG, "ants_mlp_load: NULL argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return set_error(ANTS_E_ARG, "cannot open %s", path);
  char magic[8];
  ants_mlp_cfg cfg;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "ANTSMLP1", 8) == 0 &&
            fread(&cfg, sizeof(cfg), 1, f) == 1;
  if (!ok) {
    fclose(f);
    return set_error(ANTS_E_FORMAT, "%s is not a network file", path);
  }
  ants_mlp* M = nullptr;
  ants_status st = ants_mlp_create(&cfg, &M);
  if (st != ANTS_OK) {
    fclose(f);
    return st;
  }
  std::vector<float> h((size_t)M->nparams);
  ok = fread(h.data(), sizeof(float), h.size(), f) == h.size();
  fclose(f);
  if (!ok) {
    delete M;
    return set_error(ANTS_E_FORMAT, "%s is truncated", path);
  }
  st = ants_mlp_set_params(M, h.data(), M->nparams);
  if (st != ANTS_OK) {
    delete M;
    return st;
  }
  *out = M;
  return ANTS_OK;
}

}  // extern "C"

namespace {

// Argument checks shared by both seeded entry points; fills Gr and Gf.
ants_status seeded_check(ants_lrfset* S, ants_mlp* M, const ants_grid_cfg* refine,
                         const ants_grid_cfg* fallback, double chi2ndf_max, int64_t n,
                         const float* d_signals, const float* d_seeds, const ants_out& out,
                         GridP* Gr, GridP* Gf) {
  if (!S || !refine || !fallback) return set_error(ANTS_E_ARG, "NULL set or grid configuration");
  if (!d_seeds) {
    ants_status st = check_pair(M, S);
    if (st != ANTS_OK) return st;
  }
  if (refine->start != ANTS_START_SEED)
    return set_error(ANTS_E_ARG, "the refinement grid must start at the seed");
  if (fallback->start == ANTS_START_SEED)
    return set_error(ANTS_E_ARG, "the fallback grid cannot start at the seed");
  if (!(chi2ndf_max >= 0.0))
    return set_error(ANTS_E_ARG, "chi2ndf_max must be >= 0 (0: every event falls back)");
  if (n < 0 || n > ((int64_t)1 << 31) - 1) return set_error(ANTS_E_ARG, "n_events out of range");
  ants_status st = grid_params(S->d, refine, Gr);
  if (st != ANTS_OK) return st;
  st = grid_params(S->d, fallback, Gf);
  if (st != ANTS_OK) return st;
  apply_grid_plan(S, refine, Gr);
  apply_grid_plan(S, fallback, Gf);
  if (n == 0) return ANTS_OK;
  if (!d_signals || !out.x || !out.y || !out.z || !out.E || !out.lnl || !out.chi2 || !out.ndf ||
      !out.status)
    return set_error(ANTS_E_ARG, "NULL signal or output pointer");
  int dev = 0;
  hipGetDevice(&dev);
  if (dev != S->device) return set_error(ANTS_E_ARG, "LRF set lives on another device");
  return ANTS_OK;
}

// The seeded path on caller-provided workspace: count (one int32, cleared
// here by a fill kernel), list [n] int32, seeds_ws [n][4] FP32 (unused when
// d_seeds is given).  Allocates nothing.
hipError_t seeded_run(ants_lrfset* S, ants_mlp* M, GridP Gr, GridP Gf, double chi2ndf_max,
                      int64_t n, const float* d_signals, const float* d_seeds, const ants_out& out,
                      int32_t* d_n_fallback, hipStream_t s, int32_t* count, int32_t* list,
                      float* seeds_ws) {
  hipError_t e = hipSuccess;
  const float* seeds = d_seeds;
  if (!seeds) {
    e = infer(M, S, d_signals, n, seeds_ws, true, s);
    seeds = seeds_ws;
  }
  if (e == hipSuccess) e = launch_fill_i32(count, 0, 1, s);
  IoP io;
  memset(&io, 0, sizeof(io));
  io.sig = d_signals;
  io.ld = S->ns;
  io.seeds = seeds;
  io.x = out.x;
  io.y = out.y;
  io.z = out.z;
  io.E = out.E;
  io.lnl = out.lnl;
  io.chi2 = out.chi2;
  io.ndf = out.ndf;
  io.status = out.status;
  io.path = nullptr;
  io.nfp = out.n_fp64;
  io.n = n;
  io.fb_list = list;
  io.fb_count = count;
  Gr.fb_thr = chi2ndf_max;
  if (e == hipSuccess) e = launch_grid(S->d, Gr, io, s, num_cu() * 8);
  // fallback pass over the listed events
  IoP io2 = io;
  io2.seeds = nullptr;
  io2.list = list;
  io2.list_n = count;
  io2.fb_list = nullptr;
  io2.fb_count = nullptr;
  io2.nfp = nullptr;
  Gf.or_status = ANTS_EV_FALLBACK;
  if (e == hipSuccess) e = launch_grid(S->d, Gf, io2, s, num_cu() * 8);
  if (e == hipSuccess && d_n_fallback) e = launch_copy_i32(count, d_n_fallback, 1, s);
  return e;
}

// Workspace of the allocation-free seeded entry point: one fixed array per
// device, [counter, padded to 256 B][list: kNoAllocMax int32][seeds:
// kNoAllocMax x 4 FP32].  In host code `scratch` names a host-side stand-in;
// its device address comes from hipGetSymbolAddress, once per device.
constexpr int64_t kNoAllocMax = ANTS_NOALLOC_MAX_EVENTS;
constexpr size_t kScratchList = 256;
constexpr size_t kScratchSeeds = kScratchList + (size_t)kNoAllocMax * 4;
constexpr size_t kScratchBytes = kScratchSeeds + (size_t)kNoAllocMax * 16;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array (looked up once per device)
hipError_t scratch_ptr(int dev, unsigned char** p) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* q = nullptr;
    hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!q) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = q;
  }
  *p = (unsigned char*)g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

ants_status ants_reconstruct_seeded(ants_lrfset* S, ants_mlp* M, const ants_grid_cfg* refine,
                                    const ants_grid_cfg* fallback, double chi2ndf_max,
                                    int64_t n, const float* d_signals, const float* d_seeds,
                                    ants_out out, int32_t* d_n_fallback, void* hip_stream) {
  GridP Gr, Gf;
  ants_status st = seeded_check(S, M, refine, fallback, chi2ndf_max, n, d_signals, d_seeds, out,
                                &Gr, &Gf);
  if (st != ANTS_OK || n == 0) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  hipError_t e = hipSuccess;
  if (!S->ws_count) e = hipMalloc((void**)&S->ws_count, 16);
  if (e == hipSuccess) e = ensure(&S->ws_list, &S->ws_list_bytes, (size_t)n * 4);
  if (!d_seeds && e == hipSuccess) e = ensure(&S->ws_seeds, &S->ws_seeds_bytes, (size_t)n * 16);
  if (e != hipSuccess) return hip_error(e, "ants_reconstruct_seeded (workspace)");
  e = seeded_run(S, M, Gr, Gf, chi2ndf_max, n, d_signals, d_seeds, out, d_n_fallback, s,
                 S->ws_count, (int32_t*)S->ws_list, (float*)S->ws_seeds);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_reconstruct_seeded");
}

ants_status ants_reconstruct_seeded_noalloc(ants_lrfset* S, ants_mlp* M,
                                            const ants_grid_cfg* refine,
                                            const ants_grid_cfg* fallback, double chi2ndf_max,
                                            int64_t n, const float* d_signals,
                                            const float* d_seeds, ants_out out,
                                            int32_t* d_n_fallback, void* hip_stream) {
  GridP Gr, Gf;
  ants_status st = seeded_check(S, M, refine, fallback, chi2ndf_max, n, d_signals, d_seeds, out,
                                &Gr, &Gf);
  if (st != ANTS_OK || n == 0) return st;
  if (n > kNoAllocMax)
    return set_error(ANTS_E_ARG,
                     "ants_reconstruct_seeded_noalloc: n_events = %lld exceeds the fixed "
                     "workspace of %lld events (split the batch)",
                     (long long)n, (long long)kNoAllocMax);
  unsigned char* base = nullptr;
  hipError_t e = scratch_ptr(S->device, &base);
  if (e != hipSuccess) return hip_error(e, "ants_reconstruct_seeded_noalloc (scratch address)");
  e = seeded_run(S, M, Gr, Gf, chi2ndf_max, n, d_signals, d_seeds, out, d_n_fallback,
                 (hipStream_t)hip_stream, (int32_t*)base, (int32_t*)(base + kScratchList),
                 (float*)(base + kScratchSeeds));
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_reconstruct_seeded_noalloc");
}

}  // extern "C"
