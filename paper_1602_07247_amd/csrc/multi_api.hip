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
  int kind = 0, stat = 0, max_nn = 0, max_na = 0, btab_n = 0, per_wave = 0;
  bool nonneg = true;
};

ants_status prepare(ants_lrfset* const* S, const ants_grid_cfg* cfgs, int n_sets,
                    const ants_chunk* ch, int n_chunks, Prepared* P) {
  if (!S || !cfgs || !ch) return set_error(ANTS_E_ARG, "NULL sets, configurations or chunks");
  if (n_sets < 1 || n_sets > 64) return set_error(ANTS_E_ARG, "n_sets = %d outside 1..64", n_sets);
  if (n_chunks < 0 || n_chunks > (1 << 24))
    return set_error(ANTS_E_ARG, "n_chunks = %d out of range", n_chunks);
  int dev = 0;
  hipGetDevice(&dev);
  int tab = 0, per_wave = 0;
  for (int i = 0; i < n_sets; ++i) {
    if (!S[i]) return set_error(ANTS_E_ARG, "sets[%d] is NULL", i);
    if (S[i]->device != dev) return set_error(ANTS_E_ARG, "sets[%d] lives on another device", i);
    SetDesc d;
    memset(&d, 0, sizeof(d));
    d.L = S[i]->d;
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
    d.tab_off = tab;
    const int n = d.L.kind == ANTS_LRF_AXIAL ? d.L.ntab * d.L.nintp
                  : d.L.kind == ANTS_LRF_RZ  ? d.L.nc1 * d.L.nintp
                                             : 0;
    tab += n;
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
  if ((size_t)tab * 16 > 96 * 1024)
    return set_error(ANTS_E_UNSUPPORTED, "LRF tables of all sets exceed 96 KiB of LDS");
  P->btab_n = tab;
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

ants_status run(ants_lrfset* owner, const Prepared& P, const ants_plan& plan, ants_out out,
                int64_t limit_events, hipStream_t s) {
  if (plan.events_per_item < 1 || plan.events_per_item > 4096 || plan.blocks_per_cu < 1 ||
      plan.blocks_per_cu > 32 || (plan.table_in_lds != 0 && plan.table_in_lds != 1))
    return set_error(ANTS_E_ARG, "invalid plan {%d, %d, %d}", plan.events_per_item,
                     plan.blocks_per_cu, plan.table_in_lds);
  // chunk list truncated to `limit_events` (autotuning samples)
  std::vector<ChunkDesc> ch;
  int64_t left = limit_events;
  for (const ChunkDesc& c : P.chunks) {
    if (left <= 0) break;
    ChunkDesc d = c;
    if (d.n > left) d.n = left;
    left -= d.n;
    if (d.n > 0) ch.push_back(d);
  }
  std::vector<int32_t> prefix(ch.size() + 1, 0);
  for (size_t c = 0; c < ch.size(); ++c) {
    int64_t items = (ch[c].n + plan.events_per_item - 1) / plan.events_per_item;
    int64_t next = prefix[c] + items;
    if (next > ((int64_t)1 << 31) - 2) return set_error(ANTS_E_ARG, "too many work items");
    prefix[c + 1] = (int32_t)next;
  }
  if (ch.empty()) return ANTS_OK;
  const size_t b_sets = P.sets.size() * sizeof(SetDesc);
  const size_t b_ch = ch.size() * sizeof(ChunkDesc);
  const size_t b_pre = prefix.size() * sizeof(int32_t);
  const size_t o1 = 512, o2 = o1 + ((b_sets + 255) & ~(size_t)255),
               o3 = o2 + ((b_ch + 255) & ~(size_t)255), total = o3 + b_pre;
  std::vector<unsigned char> host(total, 0);
  memcpy(host.data() + o1, P.sets.data(), b_sets);
  memcpy(host.data() + o2, ch.data(), b_ch);
  memcpy(host.data() + o3, prefix.data(), b_pre);
  hipError_t e = ensure(&owner->ws_multi, &owner->ws_multi_bytes, total);
  unsigned char* dbase = (unsigned char*)owner->ws_multi;
  // the host staging vector dies on return: wait for the copy (it is queued
  // behind earlier work on the stream, which may still read the workspace)
  if (e == hipSuccess) e = hipMemcpyAsync(dbase, host.data(), total, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(e, "multi-detector descriptors");
  MultiP M;
  memset(&M, 0, sizeof(M));
  M.sets = (const SetDesc*)(dbase + o1);
  M.n_sets = (int)P.sets.size();
  M.chunks = (const ChunkDesc*)(dbase + o2);
  M.prefix = (const int32_t*)(dbase + o3);
  M.n_chunks = (int)ch.size();
  M.n_items = prefix.back();
  M.T = plan.events_per_item;
  M.counter = (int*)dbase;   // first 512 bytes: one work counter per XCD, 64 bytes apart
  M.out.x = out.x;
  M.out.y = out.y;
  M.out.z = out.z;
  M.out.E = out.E;
  M.out.lnl = out.lnl;
  M.out.chi2 = out.chi2;
  M.out.ndf = out.ndf;
  M.out.status = out.status;
  M.per_wave_bytes = P.per_wave;
  M.btab_n = plan.table_in_lds ? P.btab_n : 0;
  M.tab_in_lds = plan.table_in_lds;
  e = launch_fill_i32(M.counter, 0, 128, s);
  int blocks = num_cu() * plan.blocks_per_cu;
  int64_t need = ((int64_t)M.n_items + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > need) blocks = (int)(need > 0 ? need : 1);
  if (e == hipSuccess) e = launch_multi(M, P.kind, P.stat, P.max_nn, P.max_na, P.nonneg, blocks, s);
  return e == hipSuccess ? ANTS_OK : hip_error(e, "ants_reconstruct_multi launch");
}

bool outputs_ok(const ants_out& o) {
  return o.x && o.y && o.z && o.E && o.lnl && o.chi2 && o.ndf && o.status;
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
  ants_plan pl = plan ? *plan : ants_plan{32, 8, 1};
  return run(sets[0], P, pl, out, INT64_MAX, (hipStream_t)hip_stream);
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
  // scratch rows are 0 .. sample-1: rewrite chunk output offsets
  int64_t row = 0;
  for (ChunkDesc& c : P.chunks) {
    c.out_off = row;
    row += c.n;
  }
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
    return set_error(ANTS_E_DEVICE, "hipEventCreate failed");
  const int Ts[3] = {8, 32, 128}, Bs[3] = {4, 8, 16};
  double best_ms = HUGE_VAL;
  int k = 0;
  for (int lds = 1; lds >= 0 && st == ANTS_OK; --lds)
    for (int ti = 0; ti < 3 && st == ANTS_OK; ++ti)
      for (int bi = 0; bi < 3 && st == ANTS_OK; ++bi, ++k) {
        ants_plan pl{Ts[ti], Bs[bi], lds};
        st = run(sets[0], P, pl, scratch, sample_events, s);   // warm-up
        hipEventRecord(a, s);
        if (st == ANTS_OK) st = run(sets[0], P, pl, scratch, sample_events, s);
        hipEventRecord(b, s);
        hipEventSynchronize(b);
        float ms = 0.f;
        hipEventElapsedTime(&ms, a, b);
        if (host_ms) host_ms[k] = ms;
        if (st == ANTS_OK && ms < best_ms) {
          best_ms = ms;
          *best = pl;
        }
      }
  hipEventDestroy(a);
  hipEventDestroy(b);
  return st;
}

}  // extern "C"
