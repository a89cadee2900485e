// Host side of the persistent multi-detector launch and its autotuner.
#include <math.h>
#include <string.h>

#include <vector>

#include "ants_internal.h"

using namespace ants;

namespace {

struct Prepared {
  std::vector<SetDesc> sets;
  std::vector<ChunkDesc> chunks;
  std::vector<int> tab_n;   // float4 entries of each set's table
  int kind = 0, stat = 0, max_nn = 0, max_na = 0, per_wave = 0;
  bool nonneg = true;
};

// A plan with a part per set (events per work item, table in LDS) and a
// launch-wide part (resident blocks per compute unit).
struct MPlan {
  int bpc = 8;
  std::vector<int> T, lds;
};

ants_status prepare(ants_lrfset* const* S, const ants_grid_cfg* cfgs, int n_sets,
                    const ants_chunk* ch, int n_chunks, Prepared* P) {
  if (!S || !cfgs || !ch) return set_error(ANTS_E_ARG, "NULL sets, configurations or chunks");
  if (n_sets < 1 || n_sets > 64) return set_error(ANTS_E_ARG, "n_sets = %d outside 1..64", n_sets);
  if (n_chunks < 0 || n_chunks > (1 << 24))
    return set_error(ANTS_E_ARG, "n_chunks = %d out of range", n_chunks);
  int dev = 0;
  hipGetDevice(&dev);
  int per_wave = 0;
  for (int i = 0; i < n_sets; ++i) {
    if (!S[i]) return set_error(ANTS_E_ARG, "sets[%d] is NULL", i);
    if (S[i]->device != dev) return set_error(ANTS_E_ARG, "sets[%d] lives on another device", i);
    SetDesc d;
    memset(&d, 0, sizeof(d));
    d.L = S[i]->d;
    if (d.L.kind != ANTS_LRF_AXIAL && d.L.kind != ANTS_LRF_XY && d.L.kind != ANTS_LRF_RZ)
      return set_error(ANTS_E_UNSUPPORTED, "sets[%d]: composite and sliced LRFs are not "
                                           "supported by the multi-detector launch", i);
    ants_status st = grid_params(d.L, &cfgs[i], &d.G);
    if (st != ANTS_OK) return st;
    if (cfgs[i].start == ANTS_START_SEED)
      return set_error(ANTS_E_ARG, "the multi-detector launch has no seeds");
    if (i == 0) {
      P->kind = d.L.kind;
      P->stat = d.G.stat;
    } else if (d.L.kind != P->kind || d.G.stat != P->stat) {
      return set_error(ANTS_E_UNSUPPORTED, "all sets must share LRF kind and statistic");
    }
    P->tab_n.push_back(d.L.kind == ANTS_LRF_AXIAL ? d.L.ntab * d.L.nintp
                       : d.L.kind == ANTS_LRF_RZ  ? d.L.nc1 * d.L.nintp
                                                  : 0);
    P->nonneg = P->nonneg && d.L.nonneg;
    P->max_nn = d.G.nn > P->max_nn ? d.G.nn : P->max_nn;
    P->max_na = d.L.na > P->max_na ? d.L.na : P->max_na;
    P->sets.push_back(d);
  }
  // every set's wave area is laid out with the launch's node-tile count
  for (const SetDesc& d : P->sets) {
    const int pw = wave_lds_bytes(d.L.kind, d.L.na, d.G.nz, d.L.nintp, d.L.nc0,
                                  node_tiles(P->max_nn));
    per_wave = pw > per_wave ? pw : per_wave;
  }
  P->per_wave = (per_wave + 15) & ~15;
  for (int c = 0; c < n_chunks; ++c) {
    if (ch[c].set < 0 || ch[c].set >= n_sets)
      return set_error(ANTS_E_ARG, "chunk %d: set %d out of range", c, ch[c].set);
    if (ch[c].n_events < 0 || ch[c].out_offset < 0)
      return set_error(ANTS_E_ARG, "chunk %d: negative size or offset", c);
    if (ch[c].n_events > 0 && !ch[c].d_signals)
      return set_error(ANTS_E_ARG, "chunk %d: NULL signals", c);
    ChunkDesc d;
    memset(&d, 0, sizeof(d));
    d.sig = ch[c].d_signals;
    d.n = ch[c].n_events;
    d.out_off = ch[c].out_offset;
    d.set = ch[c].set;
    P->chunks.push_back(d);
  }
  return ANTS_OK;
}

ants_status check_plan(const MPlan& pl) {
  if (pl.bpc < 1 || pl.bpc > 32) return set_error(ANTS_E_ARG, "blocks_per_cu = %d outside 1..32", pl.bpc);
  for (size_t i = 0; i < pl.T.size(); ++i)
    if (pl.T[i] < 1 || pl.T[i] > 4096 || (pl.lds[i] != 0 && pl.lds[i] != 1))
      return set_error(ANTS_E_ARG, "invalid plan for set %zu: {%d events, lds %d}", i, pl.T[i],
                       pl.lds[i]);
  return ANTS_OK;
}

// Descriptors of `ch` under plan `pl` copied to the device workspace of
// `owner`, stream-ordered: the pinned staging is reused only after the copy
// that last read it has finished (an event, not a stream synchronisation).
ants_status upload(ants_lrfset* owner, const Prepared& P, const MPlan& pl,
                   const std::vector<ChunkDesc>& ch, ants_out out, hipStream_t s, MultiP* M) {
  std::vector<SetDesc> sets = P.sets;
  int tab = 0, tmin = 4096;
  for (size_t i = 0; i < sets.size(); ++i) {
    sets[i].T = pl.T[i];
    tmin = pl.T[i] < tmin ? pl.T[i] : tmin;
    sets[i].tab_off = -1;
    if (pl.lds[i] && P.tab_n[i] > 0) {
      sets[i].tab_off = tab;
      tab += P.tab_n[i];
    }
  }
  if ((size_t)tab * 16 > 96 * 1024)
    return set_error(ANTS_E_UNSUPPORTED, "LRF tables staged in LDS exceed 96 KiB");
  std::vector<int32_t> prefix(ch.size() + 1, 0);
  for (size_t c = 0; c < ch.size(); ++c) {
    const int T = pl.T[ch[c].set];
    int64_t next = prefix[c] + (ch[c].n + T - 1) / T;
    if (next > ((int64_t)1 << 31) - 2) return set_error(ANTS_E_ARG, "too many work items");
    prefix[c + 1] = (int32_t)next;
  }
  const size_t b_sets = sets.size() * sizeof(SetDesc);
  const size_t b_ch = ch.size() * sizeof(ChunkDesc);
  const size_t b_pre = prefix.size() * sizeof(int32_t);
  const size_t o1 = 512, o2 = o1 + ((b_sets + 255) & ~(size_t)255),
               o3 = o2 + ((b_ch + 255) & ~(size_t)255), total = o3 + b_pre;
  hipError_t e = hipSuccess;
  if (!owner->ms_copied) e = hipEventCreateWithFlags(&owner->ms_copied, hipEventDisableTiming);
  // the previous call's copy from the staging must be done before reuse
  if (e == hipSuccess) e = hipEventSynchronize(owner->ms_copied);
  if (e == hipSuccess && owner->ms_host_bytes < total) {
    if (owner->ms_host) (void)hipHostFree(owner->ms_host);
    owner->ms_host = nullptr;
    owner->ms_host_bytes = 0;
    e = hipHostMalloc(&owner->ms_host, total, hipHostMallocDefault);
    if (e == hipSuccess) owner->ms_host_bytes = total;
  }
  if (e == hipSuccess) e = ensure(&owner->ws_multi, &owner->ws_multi_bytes, total);
  if (e != hipSuccess) return hip_error(e, "multi-detector workspace");
  unsigned char* host = (unsigned char*)owner->ms_host;
  memset(host, 0, o1);
  memcpy(host + o1, sets.data(), b_sets);
  memcpy(host + o2, ch.data(), b_ch);
  memcpy(host + o3, prefix.data(), b_pre);
  unsigned char* dbase = (unsigned char*)owner->ws_multi;
  e = hipMemcpyAsync(dbase, host, total, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipEventRecord(owner->ms_copied, s);
  if (e != hipSuccess) return hip_error(e, "multi-detector descriptors");
  memset(M, 0, sizeof(*M));
  M->sets = (const SetDesc*)(dbase + o1);
  M->n_sets = (int)sets.size();
  M->chunks = (const ChunkDesc*)(dbase + o2);
  M->prefix = (const int32_t*)(dbase + o3);
  M->n_chunks = (int)ch.size();
  M->n_items = prefix.back();
  M->xg = tmin >= 32 ? 1 : 32 / tmin;
  M->counter = (int*)dbase;   // first 512 bytes: one work counter per XCD, 64 bytes apart
  M->out.x = out.x;
  M->out.y = out.y;
  M->out.z = out.z;
  M->out.E = out.E;
  M->out.lnl = out.lnl;
  M->out.chi2 = out.chi2;
  M->out.ndf = out.ndf;
  M->out.status = out.status;
  M->per_wave_bytes = P.per_wave;
  M->btab_n = tab;
  return ANTS_OK;
}

// counters zeroed by a kernel, then the persistent launch
hipError_t launch(const Prepared& P, const MPlan& pl, const MultiP& M, hipStream_t s,
                  hipEvent_t before = nullptr, hipEvent_t after = nullptr) {
  if (M.n_chunks == 0) return hipSuccess;
  hipError_t e = launch_fill_i32(M.counter, 0, 128, s);
  int blocks = num_cu() * pl.bpc;
  int64_t need = ((int64_t)M.n_items + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > need) blocks = (int)(need > 0 ? need : 1);
  if (e == hipSuccess && before) e = hipEventRecord(before, s);
  if (e == hipSuccess) e = launch_multi(M, P.kind, P.stat, P.max_nn, P.max_na, P.nonneg, blocks, s);
  if (e == hipSuccess && after) e = hipEventRecord(after, s);
  return e;
}

bool outputs_ok(const ants_out& o) {
  return o.x && o.y && o.z && o.E && o.lnl && o.chi2 && o.ndf && o.status;
}

// the plan stored in the sets for these configurations (defaults elsewhere)
MPlan stored_plan(ants_lrfset* const* S, const ants_grid_cfg* cfgs, int n) {
  MPlan pl;
  pl.T.assign(n, 32);
  pl.lds.assign(n, 1);
  for (int i = 0; i < n; ++i)
    if (S[i]->mplan_key == grid_cfg_key(cfgs[i]) && S[i]->mplan_T > 0) {
      pl.T[i] = S[i]->mplan_T;
      pl.lds[i] = S[i]->mplan_lds;
    }
  if (S[0]->mplan_key == grid_cfg_key(cfgs[0]) && S[0]->mplan_bpc > 0) pl.bpc = S[0]->mplan_bpc;
  return pl;
}

}  // namespace

extern "C" {

ants_status ants_reconstruct_multi(ants_lrfset* const* sets, const ants_grid_cfg* cfgs,
                                   int32_t n_sets, const ants_chunk* chunks, int32_t n_chunks,
                                   const ants_plan* plan, ants_out out, void* hip_stream) {
  Prepared P;
  ants_status st = prepare(sets, cfgs, n_sets, chunks, n_chunks, &P);
  if (st != ANTS_OK) return st;
  if (!outputs_ok(out)) return set_error(ANTS_E_ARG, "an output array is NULL");
  MPlan pl;
  if (plan) {
    pl.bpc = plan->blocks_per_cu;
    pl.T.assign(n_sets, plan->events_per_item);
    pl.lds.assign(n_sets, plan->table_in_lds);
  } else {
    pl = stored_plan(sets, cfgs, n_sets);
  }
  st = check_plan(pl);
  if (st != ANTS_OK) return st;
  std::vector<ChunkDesc> ch;
  for (const ChunkDesc& c : P.chunks)
    if (c.n > 0) ch.push_back(c);
  if (ch.empty()) return ANTS_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  MultiP M;
  st = upload(sets[0], P, pl, ch, out, s, &M);
  if (st != ANTS_OK) return st;
  hipError_t e = launch(P, pl, M, s);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_reconstruct_multi launch");
}

ants_status ants_autotune_multi(ants_lrfset* const* sets, const ants_grid_cfg* cfgs,
                                int32_t n_sets, const ants_chunk* chunks, int32_t n_chunks,
                                int64_t sample_events, ants_out scratch, ants_plan* best,
                                double* host_ms, void* hip_stream) {
  Prepared P;
  ants_status st = prepare(sets, cfgs, n_sets, chunks, n_chunks, &P);
  if (st != ANTS_OK) return st;
  if (!best || !outputs_ok(scratch) || sample_events < 1)
    return set_error(ANTS_E_ARG, "autotune needs outputs, a plan pointer and a sample > 0");
  hipStream_t s = (hipStream_t)hip_stream;
  // sample: whole chunks taken at an even stride through the stream (every
  // detector in proportion), written to scratch rows 0 .. sample-1
  int64_t total = 0;
  for (const ChunkDesc& c : P.chunks) total += c.n;
  std::vector<ChunkDesc> ch;
  if (total > 0) {
    const double stride = (double)total / (double)(sample_events < total ? sample_events : total);
    int64_t row = 0, pos = 0;
    double next = 0.0;
    for (const ChunkDesc& c : P.chunks) {
      if (c.n > 0 && (double)pos + (double)c.n > next && row < sample_events) {
        ChunkDesc d = c;
        if (d.n > sample_events - row) d.n = sample_events - row;
        d.out_off = row;
        row += d.n;
        ch.push_back(d);
        next += (double)c.n * stride;
      }
      pos += c.n;
    }
  }
  if (ch.empty()) return set_error(ANTS_E_ARG, "autotune: no events in the chunk list");
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return set_error(ANTS_E_DEVICE, "hipEventCreate failed");
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    return set_error(ANTS_E_DEVICE, "hipEventCreate failed");
  }
  int k = 0;
  // one candidate: descriptors uploaded, a warm-up launch, then the kernel
  // alone timed between events on the stream
  auto time_plan = [&](const MPlan& pl, float* ms) -> ants_status {
    MultiP M;
    ants_status r = upload(sets[0], P, pl, ch, scratch, s, &M);
    if (r != ANTS_OK) return r;
    hipError_t e = launch(P, pl, M, s);
    if (e == hipSuccess) e = launch(P, pl, M, s, a, b);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (e != hipSuccess) return hip_error(e, "ants_autotune_multi");
    if (host_ms) host_ms[k] = *ms;
    ++k;
    return ANTS_OK;
  };
  MPlan cur;
  cur.T.assign(n_sets, 32);
  cur.lds.assign(n_sets, 1);
  float best_ms = HUGE_VALF;
  // stage 1: resident blocks per compute unit
  const int Bs[3] = {4, 8, 16};
  int bpc = 8;
  for (int bi = 0; bi < 3 && st == ANTS_OK; ++bi) {
    MPlan pl = cur;
    pl.bpc = Bs[bi];
    float ms = 0.f;
    st = time_plan(pl, &ms);
    if (st == ANTS_OK && ms < best_ms) {
      best_ms = ms;
      bpc = Bs[bi];
    }
  }
  cur.bpc = bpc;
  // stage 2: each set in turn, events per item x table in LDS, the other
  // sets at their current choice
  const int Ts[3] = {8, 32, 128};
  for (int i = 0; i < n_sets && st == ANTS_OK; ++i)
    for (int lds = 1; lds >= 0 && st == ANTS_OK; --lds)
      for (int ti = 0; ti < 3 && st == ANTS_OK; ++ti) {
        MPlan pl = cur;
        pl.T[i] = Ts[ti];
        pl.lds[i] = lds;
        float ms = 0.f;
        st = time_plan(pl, &ms);
        if (st == ANTS_OK && ms < best_ms) {
          best_ms = ms;
          cur = pl;
        }
      }
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (st != ANTS_OK) return st;
  for (int i = 0; i < n_sets; ++i) {
    sets[i]->mplan_key = grid_cfg_key(cfgs[i]);
    sets[i]->mplan_T = cur.T[i];
    sets[i]->mplan_lds = cur.lds[i];
    sets[i]->mplan_bpc = cur.bpc;
  }
  *best = ants_plan{cur.T[0], cur.bpc, cur.lds[0]};
  return ANTS_OK;
}

}  // extern "C"
