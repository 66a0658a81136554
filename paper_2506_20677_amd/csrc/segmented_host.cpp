// Host side of the batched segmented sort: the blocking and the
// enqueue-only entry points, hipGraph capture of the enqueue-only form, and
// the autotuner that picks the LDS kernel variant of every size class.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <vector>

#include "segmented.hpp"
#include "ss_host.hpp"

namespace ahs {
namespace {

struct SegLayout {
  size_t queues = 0, large = 0, large_ids = 0, bounds = 0, partial = 0, segctr = 0, status = 0;
  size_t linfo = 0, hsegs = 0, hlarge = 0, hslot_of = 0, hslots = 0, rsegs = 0, rinfo = 0, rdig = 0, dctr = 0;
  size_t total = 0;
  uint64_t chunk_cap = 0, lcap = 0, slot_cap = 0, unit_cap = 0, tile_cap = 0;
};

SegLayout seg_layout(size_t base, uint64_t n_total, uint32_t nseg, int key_bytes, int with_payload) {
  SegLayout L;
  size_t o = base;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.queues = take(4 * (size_t)SEG_NCLASS * ((size_t)nseg + 1));
  L.large = take(sizeof(SsSeg) * ((size_t)nseg + 1));
  L.large_ids = take(4 * ((size_t)nseg + 1));
  L.bounds = take(8 * ((size_t)nseg + 1));
  L.chunk_cap = n_total / SEG_CH + (uint64_t)nseg + 1;
  L.partial = take(sizeof(double) * L.chunk_cap);
  L.segctr = take(sizeof(SegCounters) + 2 * sizeof(SsCounters));
  L.status = take(256);
  // large-segment dispatch: a large segment holds more than SS_CAP keys
  L.lcap = std::min<uint64_t>(nseg, n_total / (SS_CAP + 1)) + 1;
  L.slot_cap = n_total / (SEG_HU + 1) + 1;
  L.unit_cap = n_total / SEG_HU_MULTI + L.lcap;
  L.tile_cap = n_total / seg_radix_tile(key_bytes, with_payload, 0) + L.lcap;
  L.linfo = take(sizeof(SegLarge) * ((size_t)nseg + 1));
  L.hsegs = take(sizeof(SsSeg) * L.lcap);
  L.hlarge = take(4 * L.lcap);
  L.hslot_of = take(4 * L.lcap);
  L.hslots = take(4 * 65536 * (size_t)L.slot_cap);
  L.rsegs = take(sizeof(SsSeg) * L.lcap);
  L.rinfo = take(sizeof(SegRadixInfo) * L.lcap);
  L.rdig = take(4 * 8 * 256 * (size_t)L.lcap);
  L.dctr = take(sizeof(SegDispatchCounters));
  L.total = o;
  return L;
}

int key_bytes_of(ahs_dtype d) { return (d == AHS_U32 || d == AHS_F32 || d == AHS_I32) ? 4 : 8; }

// One batched call: arguments checked, tables placed, SegArgs filled.
struct SegCall {
  SortJob j;
  SsLayout S;
  SsTables T;
  SegLayout G;
  SegArgs a;
  SegDispatchArgs d;
  SegCounters* sctr;
  SsCounters* rec0;        // level 0 of the sample sort
  SsCounters* rec_chunks;  // chunks of the large segments
  uint32_t nseg;
  int pay;
};

ahs_status seg_setup(SegCall& C, ahs_context* ctx, const void* d_keys_in, void* d_keys_out, const uint32_t* d_vals_in,
                     uint32_t* d_vals_out, const uint64_t* d_offsets, uint32_t nseg, uint64_t n_total,
                     ahs_dtype dtype, ahs_strategy requested, const ahs_config* cfg, void* d_ws, size_t ws_bytes,
                     void* stream, uint8_t* d_chosen, ahs_feature_vector* d_feats) {
  if (!ctx) return AHS_E_INVALID_ARG;
  if ((int)dtype < 0 || (int)dtype > (int)AHS_I64) return ctx->fail(AHS_E_INVALID_ARG, "bad dtype");
  if ((int)requested < AHS_AUTO || (int)requested > AHS_QUICK)
    return ctx->fail(AHS_E_INVALID_ARG, "strategy %d cannot be requested", (int)requested);
  if ((d_vals_in == nullptr) != (d_vals_out == nullptr))
    return ctx->fail(AHS_E_INVALID_ARG, "payload pointers must be both null or both set");
  ahs_config c;
  if (cfg) c = *cfg; else ahs_config_init(&c, AHS_PRESET_GPU);
  if (c.use_model) return ctx->fail(AHS_E_UNSUPPORTED, "the batched sort does not evaluate the model");
  if (c.k_count == 0) return ctx->fail(AHS_E_INVALID_ARG, "k_count must be positive");
  if (!d_offsets || !d_ws || (n_total && (!d_keys_in || !d_keys_out)))
    return ctx->fail(AHS_E_INVALID_ARG, "null device pointer");
  const int kb = key_bytes_of(dtype);
  if (d_keys_in != d_keys_out) {
    const uintptr_t x = (uintptr_t)d_keys_in, y = (uintptr_t)d_keys_out;
    if (x < y + kb * n_total && y < x + kb * n_total)
      return ctx->fail(AHS_E_INVALID_ARG, "input and output partially overlap");
  }
  SortJob& j = C.j;
  j.ctx = ctx;
  j.kk = (int)dtype;
  j.key_bytes = kb;
  j.kin = d_keys_in;
  j.kout = d_keys_out;
  j.vin = d_vals_in;
  j.vout = d_vals_out;
  j.n = n_total;
  j.ws = d_ws;
  j.s = (hipStream_t)stream;
  j.L = plan_layout(n_total, kb, d_vals_in ? 1 : 0, true);
  memset(&j.f, 0, sizeof j.f);
  C.G = seg_layout(j.L.total, n_total, nseg, kb, d_vals_in ? 1 : 0);
  if (ws_bytes < C.G.total) return ctx->fail(AHS_E_WORKSPACE, "workspace %zu < %zu", ws_bytes, C.G.total);
  AHS_HIP(j, hipSetDevice(ctx->device), "set device");
  C.S = ss_layout(n_total, kb);
  C.T = ss_tables(j, C.S);
  C.sctr = at<SegCounters>(d_ws, C.G.segctr);
  C.rec0 = reinterpret_cast<SsCounters*>(C.sctr + 1);
  C.rec_chunks = C.rec0 + 1;
  C.nseg = nseg;
  C.pay = d_vals_in != nullptr;
  SegArgs& a = C.a;
  a.kin = d_keys_in;
  a.kout = d_keys_out;
  a.vin = d_vals_in;
  a.vout = d_vals_out;
  a.offs = d_offsets;
  a.queues = at<uint32_t>(d_ws, C.G.queues);
  a.qcap = nseg + 1;
  a.large = at<SsSeg>(d_ws, C.G.large);
  a.large_ids = at<uint32_t>(d_ws, C.G.large_ids);
  a.ctr = C.sctr;
  a.chunks = C.rec_chunks;
  a.chunk_cap = (uint32_t)std::min<uint64_t>(C.G.chunk_cap, 0xFFFFFFFFull);
  a.bounds = at<uint32_t>(d_ws, C.G.bounds);
  a.partial = at<double>(d_ws, C.G.partial);
  a.cfg.n_small = c.n_small;
  a.cfg.k_count = c.k_count;
  a.cfg.k_radix = c.k_radix;
  a.cfg.h_ratio = c.h_ratio;
  a.requested = (uint32_t)requested;
  a.chosen = d_chosen;
  a.feats = reinterpret_cast<DevFeatures*>(d_feats);

  SegDispatchArgs& d = C.d;
  d.kin = d_keys_in;
  d.kout = d_keys_out;
  d.ktmp = at<void>(d_ws, j.L.tmpk);
  d.vin = d_vals_in;
  d.vout = d_vals_out;
  d.vtmp = d_vals_in ? at<uint32_t>(d_ws, j.L.tmpv) : nullptr;
  d.large = a.large;
  d.large_ids = a.large_ids;
  d.ctr = C.sctr;
  d.chunks = C.rec_chunks;
  d.chunk_cap = a.chunk_cap;
  d.linfo = at<SegLarge>(d_ws, C.G.linfo);
  d.qsegs = C.T.segs[0];
  d.qrec = C.rec0;
  d.qcap = (uint32_t)std::min<uint64_t>(C.S.seg_cap, 0xFFFFFFFFull);
  d.hsegs = at<SsSeg>(d_ws, C.G.hsegs);
  d.hlarge = at<uint32_t>(d_ws, C.G.hlarge);
  d.hslots = at<uint32_t>(d_ws, C.G.hslots);
  d.hslot_of = at<uint32_t>(d_ws, C.G.hslot_of);
  d.slot_cap = (uint32_t)C.G.slot_cap;
  d.rsegs = at<SsSeg>(d_ws, C.G.rsegs);
  d.rinfo = at<SegRadixInfo>(d_ws, C.G.rinfo);
  d.rdig = at<uint32_t>(d_ws, C.G.rdig);
  d.list_cap = (uint32_t)C.G.lcap;
  d.tile_cap = (uint32_t)std::min<uint64_t>(C.G.tile_cap, 0xFFFFFFFFull);
  d.unit_cap = (uint32_t)std::min<uint64_t>(C.G.unit_cap, 0xFFFFFFFFull);
  d.dctr = at<SegDispatchCounters>(d_ws, C.G.dctr);
  d.status = C.T.status;  // the radix passes and the sample-sort levels run one after the other
  d.cfg = a.cfg;
  d.requested = a.requested;
  d.in_place = (d_keys_in == d_keys_out || (d_vals_in && d_vals_in == d_vals_out)) ? 1u : 0u;
  d.chosen = d_chosen;
  // the radix passes' look-back words live in the sample sort's status table
  if ((uint64_t)C.G.tile_cap * 256 * 8 > 8ull * SS_NB * C.S.tile_cap)
    return ctx->fail(AHS_E_DEVICE, "radix status table exceeds the sample sort's");
  return AHS_OK;
}

// Counters cleared, segments classified into the size-class queues and the
// large list, level 0 of the sample sort numbered.  Enqueue only.
ahs_status seg_classify(SegCall& C, uint64_t n_total) {
  SortJob& j = C.j;
  AHS_HIP(j,
          launch_fill_u32(reinterpret_cast<uint32_t*>(C.sctr), (sizeof(SegCounters) + 2 * sizeof(SsCounters)) / 4,
                          0u, j.s),
          "fill");
  static_assert(sizeof(SegDispatchCounters) % 4 == 0, "counters fill as words");
  AHS_HIP(j, launch_fill_u32(reinterpret_cast<uint32_t*>(C.d.dctr), sizeof(SegDispatchCounters) / 4, 0u, j.s),
          "fill");
  {
    ProfScope p(j.ctx, "seg_classify", j.s);
    AHS_HIP(j,
            launch_seg_classify(C.a.offs, C.nseg, n_total, const_cast<uint32_t*>(C.a.queues), C.a.qcap, C.d.linfo,
                                const_cast<SsSeg*>(C.a.large), const_cast<uint32_t*>(C.a.large_ids), C.sctr, j.s),
            "classify");
  }
  AHS_HIP(j, launch_seg_gate(C.sctr, C.rec_chunks, j.s), "gate");
  AHS_HIP(j, launch_ss_tiles(const_cast<SsSeg*>(C.a.large), C.rec_chunks, SEG_CH, C.nseg + 1, j.s), "chunks");
  return AHS_OK;
}

ahs_status seg_small_all(SegCall& C, const uint32_t* exact_counts, double small_bytes) {
  SortJob& j = C.j;
  ProfScope p(j.ctx, "seg_small", j.s, small_bytes);
  for (int cls = 0; cls < SEG_NCLASS; ++cls) {
    const int v = j.ctx->seg_variant[j.kk][C.pay][cls];
    uint32_t grid;
    if (exact_counts) {
      grid = exact_counts[cls];
    } else {
      const uint32_t res = seg_small_resident(j.kk, C.pay, v, j.ctx->cu_count);
      grid = std::min<uint32_t>(C.nseg, res);
    }
    AHS_HIP(j, launch_seg_small(j.kk, C.pay, C.a, cls, v, grid, j.s), "small segments");
  }
  return AHS_OK;
}

// Large segments: min/max, decisions (entropy where the span calls for it),
// the radix list's digit passes, then the quick list's sample-sort levels
// (device-driven: `levels` of them; host-driven when levels < 0), and the
// features of the sorted segments when the caller asked for them.
ahs_status seg_large_all(SegCall& C, uint64_t max_seg, int levels) {
  SortJob& j = C.j;
  const uint32_t cu = j.ctx->cu_count ? j.ctx->cu_count : 256;
  const int variant = j.ctx->seg_radix_variant[j.kk][C.pay];
  {
    ProfScope p(j.ctx, "seg_dispatch", j.s);
    AHS_HIP(j, launch_seg_dispatch(j.kk, C.d, cu, j.s), "large-segment decisions");
  }
  AHS_HIP(j, launch_ss_tiles(C.T.segs[0], C.rec0, (uint32_t)ss_tile(j.key_bytes), (uint32_t)C.S.seg_cap, j.s),
          "tiles");
  {
    ProfScope p(j.ctx, "seg_radix_digits", j.s);
    AHS_HIP(j, launch_seg_radix_prepare(j.kk, C.d, seg_radix_tile(j.key_bytes, C.pay, variant), cu, j.s),
            "radix digit counts");
  }
  const int npass = j.key_bytes == 4 ? 5 : SEG_MAX_PASSES;  // digits, plus a repeated first pass in place
  for (int q = 0; q < npass; ++q) {
    ProfScope p(j.ctx, "seg_radix_pass", j.s);
    AHS_HIP(j, launch_seg_radix_pass(j.kk, C.pay, variant, C.d, q, max_seg, cu, j.s), "radix pass");
  }
  if (levels > 0) {
    AHS_TRY(ss_levels_device(j, C.S, C.T, C.rec0, levels, max_seg));
  } else if (levels < 0) {
    char* pin = static_cast<char*>(j.ctx->pinned);
    AHS_HIP(j, hipMemcpyAsync(pin, C.rec0, sizeof(SsCounters), hipMemcpyDeviceToHost, j.s), "copy");
    AHS_HIP(j, hipMemcpyAsync(pin + 64, C.d.dctr, sizeof(SegDispatchCounters), hipMemcpyDeviceToHost, j.s), "copy");
    AHS_HIP(j, hipStreamSynchronize(j.s), "synchronize");
    SsCounters q;
    SegDispatchCounters dc;
    memcpy(&q, pin, sizeof q);
    memcpy(&dc, pin + 64, sizeof dc);
    if (dc.bad) return j.ctx->fail(AHS_E_DEVICE, "batched sort table overflow");
    if (q.nsegs_next) AHS_TRY(ss_levels_host(j, C.S, C.T, q.nsegs_next, q.ntiles_next, q.seg_keys_next, max_seg));
  }
  if (C.a.feats) {
    ProfScope p(j.ctx, "seg_large_features", j.s);
    const uint32_t lmax = (uint32_t)std::min<uint64_t>(C.nseg, j.n / (SS_CAP + 1) + 1);
    AHS_HIP(j,
            launch_seg_large(j.kk, C.a, (lmax + 63) / 64, seg_chunk_resident(j.kk, cu),
                             std::min<uint32_t>(lmax, 2 * cu), j.s),
            "large-segment features");
  }
  return AHS_OK;
}

ahs_status seg_enqueue_async(SegCall& C, uint64_t n_total, uint64_t max_seg_hint, uint32_t* d_status) {
  SortJob& j = C.j;
  AHS_TRY(seg_classify(C, n_total));
  AHS_TRY(seg_small_all(C, nullptr, 0.0));
  uint64_t max_seg = max_seg_hint ? std::min<uint64_t>(max_seg_hint, n_total) : n_total;
  if (max_seg > 0xFFFFFFFFull) max_seg = 0xFFFFFFFFull;
  const int levels = C.nseg ? ss_levels_for(max_seg) : 0;
  if (C.nseg && max_seg > (uint64_t)SS_CAP) AHS_TRY(seg_large_all(C, max_seg, levels));
  AHS_HIP(j, launch_seg_status(C.sctr, C.T.ctr, levels, C.d.dctr, max_seg, d_status, j.s), "status");
  return AHS_OK;
}

}  // namespace
}  // namespace ahs

using namespace ahs;

extern "C" size_t ahs_segmented_workspace_bytes(uint64_t n_total, uint32_t nseg, ahs_dtype dtype, int with_payload) {
  if ((int)dtype < 0 || (int)dtype > (int)AHS_I64) return 0;
  const Layout L = plan_layout(n_total, key_bytes_of(dtype), with_payload ? 1 : 0, true);
  return seg_layout(L.total, n_total, nseg, key_bytes_of(dtype), with_payload ? 1 : 0).total;
}

extern "C" ahs_status ahs_sort_segmented(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                                         const uint32_t* d_vals_in, uint32_t* d_vals_out, const uint64_t* d_offsets,
                                         uint32_t nseg, uint64_t n_total, ahs_dtype dtype, ahs_strategy requested,
                                         const ahs_config* cfg, void* d_ws, size_t ws_bytes, void* stream,
                                         uint8_t* d_chosen, ahs_feature_vector* d_feats) {
  if (ctx && nseg == 0) return AHS_OK;
  SegCall C;
  AHS_TRY(seg_setup(C, ctx, d_keys_in, d_keys_out, d_vals_in, d_vals_out, d_offsets, nseg, n_total, dtype, requested,
                    cfg, d_ws, ws_bytes, stream, d_chosen, d_feats));
  SortJob& j = C.j;
  AHS_TRY(seg_classify(C, n_total));
  char* pin = static_cast<char*>(ctx->pinned);
  AHS_HIP(j, hipMemcpyAsync(pin, C.sctr, sizeof(SegCounters), hipMemcpyDeviceToHost, j.s), "copy");
  AHS_HIP(j, hipStreamSynchronize(j.s), "synchronize");
  SegCounters sc;
  memcpy(&sc, pin, sizeof sc);
  if (sc.bad) return ctx->fail(AHS_E_INVALID_ARG, "offsets are not non-decreasing or do not end at n_total");
  const double rec_bytes = 2.0 * j.key_bytes + (C.pay ? 8.0 : 0.0);
  AHS_TRY(seg_small_all(C, sc.nclass, rec_bytes * (double)sc.small_keys));
  if (sc.nlarge) AHS_TRY(seg_large_all(C, sc.max_large, -1));
  return AHS_OK;
}

extern "C" ahs_status ahs_sort_segmented_async(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                                               const uint32_t* d_vals_in, uint32_t* d_vals_out,
                                               const uint64_t* d_offsets, uint32_t nseg, uint64_t n_total,
                                               uint64_t max_seg_hint, ahs_dtype dtype, ahs_strategy requested,
                                               const ahs_config* cfg, void* d_ws, size_t ws_bytes, void* stream,
                                               uint8_t* d_chosen, ahs_feature_vector* d_feats, uint32_t* d_status) {
  if (!ctx) return AHS_E_INVALID_ARG;
  if (!d_status) return ctx->fail(AHS_E_INVALID_ARG, "d_status is required");
  SegCall C;
  AHS_TRY(seg_setup(C, ctx, d_keys_in, d_keys_out, d_vals_in, d_vals_out, d_offsets, nseg, n_total, dtype, requested,
                    cfg, d_ws, ws_bytes, stream, d_chosen, d_feats));
  return seg_enqueue_async(C, n_total, max_seg_hint, d_status);
}

struct ahs_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int device = 0;
};

extern "C" ahs_status ahs_sort_segmented_capture(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                                                 const uint32_t* d_vals_in, uint32_t* d_vals_out,
                                                 const uint64_t* d_offsets, uint32_t nseg, uint64_t n_total,
                                                 uint64_t max_seg_hint, ahs_dtype dtype, ahs_strategy requested,
                                                 const ahs_config* cfg, void* d_ws, size_t ws_bytes,
                                                 uint8_t* d_chosen, ahs_feature_vector* d_feats, uint32_t* d_status,
                                                 ahs_graph** out) {
  if (!ctx || !out) return AHS_E_INVALID_ARG;
  *out = nullptr;
  if (!d_status) return ctx->fail(AHS_E_INVALID_ARG, "d_status is required");
  if (ctx->check(hipSetDevice(ctx->device), "set device") != AHS_OK) return AHS_E_DEVICE;
  hipStream_t cs = nullptr;
  if (ctx->check(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "stream") != AHS_OK) return AHS_E_DEVICE;
  SegCall C;
  ahs_status st = seg_setup(C, ctx, d_keys_in, d_keys_out, d_vals_in, d_vals_out, d_offsets, nseg, n_total, dtype,
                            requested, cfg, d_ws, ws_bytes, cs, d_chosen, d_feats);
  if (st != AHS_OK) {
    (void)hipStreamDestroy(cs);
    return st;
  }
  hipGraph_t g = nullptr;
  st = ctx->check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
  if (st == AHS_OK) {
    ctx->capturing = true;
    st = seg_enqueue_async(C, n_total, max_seg_hint, d_status);
    ctx->capturing = false;
    const ahs_status st2 = ctx->check(hipStreamEndCapture(cs, &g), "end capture");
    if (st == AHS_OK) st = st2;
  }
  (void)hipStreamDestroy(cs);
  if (st != AHS_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  ahs_graph* G = new (std::nothrow) ahs_graph();
  if (!G) {
    (void)hipGraphDestroy(g);
    return ctx->fail(AHS_E_OOM, "graph handle");
  }
  G->graph = g;
  G->device = ctx->device;
  st = ctx->check(hipGraphInstantiate(&G->exec, g, nullptr, nullptr, 0), "instantiate graph");
  if (st != AHS_OK) {
    (void)hipGraphDestroy(g);
    delete G;
    return st;
  }
  *out = G;
  return AHS_OK;
}

extern "C" ahs_status ahs_graph_launch(ahs_graph* g, void* stream) {
  if (!g || !g->exec) return AHS_E_INVALID_ARG;
  if (hipSetDevice(g->device) != hipSuccess) return AHS_E_DEVICE;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? AHS_OK : AHS_E_DEVICE;
}

extern "C" void ahs_graph_destroy(ahs_graph* g) {
  if (!g) return;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
}

extern "C" ahs_status ahs_segmented_get_variants(ahs_context* ctx, ahs_dtype dtype, int with_payload, int* h_caps) {
  if (!ctx || !h_caps || (int)dtype < 0 || (int)dtype > (int)AHS_I64) return AHS_E_INVALID_ARG;
  for (int c = 0; c < SEG_NCLASS; ++c)
    h_caps[c] = (int)SEG_CLASS_CAP[ctx->seg_variant[dtype][with_payload ? 1 : 0][c]];
  return AHS_OK;
}

extern "C" ahs_status ahs_segmented_set_variants(ahs_context* ctx, ahs_dtype dtype, int with_payload,
                                                 const int* h_caps) {
  if (!ctx || !h_caps || (int)dtype < 0 || (int)dtype > (int)AHS_I64) return AHS_E_INVALID_ARG;
  int v[SEG_NCLASS];
  for (int c = 0; c < SEG_NCLASS; ++c) {
    v[c] = -1;
    for (int k = 0; k < SEG_NVARIANT; ++k)
      if ((uint32_t)h_caps[c] == SEG_CLASS_CAP[k]) v[c] = k;
    if (v[c] < c) return ctx->fail(AHS_E_INVALID_ARG, "class %d: capacity %d does not cover it", c, h_caps[c]);
  }
  for (int c = 0; c < SEG_NCLASS; ++c) ctx->seg_variant[dtype][with_payload ? 1 : 0][c] = v[c];
  return AHS_OK;
}

extern "C" ahs_status ahs_segmented_autotune(ahs_context* ctx, ahs_dtype dtype, int with_payload, void* stream,
                                             int* h_caps, double* h_ms) {
  if (!ctx || (int)dtype < 0 || (int)dtype > (int)AHS_I64) return AHS_E_INVALID_ARG;
  const int kb = key_bytes_of(dtype);
  const int pay = with_payload ? 1 : 0;
  hipStream_t s = (hipStream_t)stream;
  if (ctx->check(hipSetDevice(ctx->device), "set device") != AHS_OK) return AHS_E_DEVICE;
  // one synthetic batch per class: about 2^22 keys in segments spread over
  // the class's size range
  constexpr uint64_t KEYS = 1u << 22;
  constexpr uint32_t MAXSEG = KEYS / 512 + 1;  // smallest class lower bound is 1 key
  // the radix tile is timed on a batch large enough to keep every CU busy
  // for many tiles: on a small batch the smaller tile wins by its shorter
  // tail although it is slower per key on large batches
  constexpr uint64_t RKEYS = 1u << 26;
  const uint64_t nmax = RKEYS;
  const size_t wsb = ahs_segmented_workspace_bytes(nmax, MAXSEG * 8, dtype, pay);
  void *kin = nullptr, *kout = nullptr, *vin = nullptr, *vout = nullptr, *ws = nullptr, *offs = nullptr;
  auto release = [&]() {
    if (kin) (void)hipFree(kin);
    if (kout) (void)hipFree(kout);
    if (vin) (void)hipFree(vin);
    if (vout) (void)hipFree(vout);
    if (ws) (void)hipFree(ws);
    if (offs) (void)hipFree(offs);
  };
  bool ok = hipMalloc(&kin, kb * nmax) == hipSuccess && hipMalloc(&kout, kb * nmax) == hipSuccess &&
            hipMalloc(&ws, wsb) == hipSuccess && hipMalloc(&offs, 8 * ((size_t)MAXSEG * 8 + 1)) == hipSuccess;
  if (ok && pay) ok = hipMalloc(&vin, 4 * nmax) == hipSuccess && hipMalloc(&vout, 4 * nmax) == hipSuccess;
  if (!ok) {
    release();
    return ctx->fail(AHS_E_OOM, "autotune buffers");
  }
  ahs_status st = ctx->check(launch_tune_fill((int)dtype, kin, nmax, 0x7A11ull, s), "fill");
  if (st == AHS_OK && pay) st = ctx->check(launch_fill_u32((uint32_t*)vin, nmax, 1u, s), "fill");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const bool was_profiling = ctx->profiling;
  ctx->profiling = false;
  std::vector<uint64_t> h_offs;
  for (int cls = 0; cls < SEG_NCLASS && st == AHS_OK; ++cls) {
    const uint32_t lo = cls == 0 ? 1 : SEG_CLASS_CAP[cls - 1] + 1, hi = SEG_CLASS_CAP[cls];
    h_offs.assign(1, 0);
    for (uint32_t i = 0; h_offs.back() < KEYS; ++i)
      h_offs.push_back(h_offs.back() + lo + (uint64_t)i * 7919u % (hi - lo + 1));
    const uint32_t nseg = (uint32_t)h_offs.size() - 1;
    const uint64_t n = h_offs.back();
    st = ctx->check(hipMemcpyAsync(offs, h_offs.data(), 8 * h_offs.size(), hipMemcpyHostToDevice, s), "copy");
    if (st != AHS_OK) break;
    SegCall C;
    st = seg_setup(C, ctx, kin, kout, pay ? (const uint32_t*)vin : nullptr, pay ? (uint32_t*)vout : nullptr,
                   (const uint64_t*)offs, nseg, n, dtype, AHS_AUTO, nullptr, ws, wsb, stream, nullptr, nullptr);
    if (st == AHS_OK) st = seg_classify(C, n);
    if (st != AHS_OK) break;
    int best = -1;
    float best_ms = 0.f;
    for (int v = cls; v < SEG_NVARIANT && st == AHS_OK; ++v) {
      float ms_min = 1e30f;
      for (int rep = 0; rep < 4 && st == AHS_OK; ++rep) {  // first run warms up
        (void)hipEventRecord(e0, s);
        st = ctx->check(launch_seg_small((int)dtype, pay, C.a, cls, v, nseg, s), "tune launch");
        (void)hipEventRecord(e1, s);
        if (st != AHS_OK) break;
        st = ctx->check(hipEventSynchronize(e1), "tune sync");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) ms_min = std::min(ms_min, ms);
      }
      if (st == AHS_OK && (best < 0 || ms_min < best_ms)) {
        best = v;
        best_ms = ms_min;
      }
    }
    if (st == AHS_OK) {
      ctx->seg_variant[dtype][pay][cls] = best;
      if (h_caps) h_caps[cls] = (int)SEG_CLASS_CAP[best];
      if (h_ms) h_ms[cls] = best_ms;
    }
  }
  // the radix passes of large segments: both tile shapes on one synthetic
  // batch of large segments sorted with RADIX forced (2^26 keys in
  // segments of 2^14 .. 2^19 keys)
  if (st == AHS_OK) {
    h_offs.assign(1, 0);
    for (uint32_t i = 0; h_offs.back() < RKEYS; ++i)
      h_offs.push_back(h_offs.back() + std::min<uint64_t>(16384u << (i % 6), RKEYS - h_offs.back()));
    const uint32_t nseg = (uint32_t)h_offs.size() - 1;
    const uint64_t n = h_offs.back();
    st = ctx->check(hipMemcpyAsync(offs, h_offs.data(), 8 * h_offs.size(), hipMemcpyHostToDevice, s), "copy");
    int best = -1;
    float best_ms = 0.f;
    for (int v = 0; v < 2 && st == AHS_OK; ++v) {
      ctx->seg_radix_variant[dtype][pay] = v;
      float ms_min = 1e30f;
      for (int rep = 0; rep < 4 && st == AHS_OK; ++rep) {  // first run warms up
        SegCall C;
        st = seg_setup(C, ctx, kin, kout, pay ? (const uint32_t*)vin : nullptr, pay ? (uint32_t*)vout : nullptr,
                       (const uint64_t*)offs, nseg, n, dtype, AHS_RADIX, nullptr, ws, wsb, stream, nullptr, nullptr);
        if (st == AHS_OK) st = seg_classify(C, n);
        if (st != AHS_OK) break;
        (void)hipEventRecord(e0, s);
        st = seg_large_all(C, 16384u << 5, 0);
        (void)hipEventRecord(e1, s);
        if (st != AHS_OK) break;
        st = ctx->check(hipEventSynchronize(e1), "tune sync");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0) ms_min = std::min(ms_min, ms);
      }
      if (st == AHS_OK && (best < 0 || ms_min < best_ms)) {
        best = v;
        best_ms = ms_min;
      }
    }
    if (st == AHS_OK) ctx->seg_radix_variant[dtype][pay] = best;
  }
  ctx->profiling = was_profiling;
  if (st == AHS_OK) st = ctx->check(hipStreamSynchronize(s), "synchronize");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  release();
  return st;
}

extern "C" ahs_status ahs_segmented_get_radix_tile(ahs_context* ctx, ahs_dtype dtype, int with_payload,
                                                   uint32_t* h_keys_per_tile) {
  if (!ctx || !h_keys_per_tile || (int)dtype < 0 || (int)dtype > (int)AHS_I64) return AHS_E_INVALID_ARG;
  const int pay = with_payload ? 1 : 0;
  *h_keys_per_tile = seg_radix_tile(key_bytes_of(dtype), pay, ctx->seg_radix_variant[dtype][pay]);
  return AHS_OK;
}

extern "C" ahs_status ahs_segmented_set_radix_tile(ahs_context* ctx, ahs_dtype dtype, int with_payload,
                                                   uint32_t keys_per_tile) {
  if (!ctx || (int)dtype < 0 || (int)dtype > (int)AHS_I64) return AHS_E_INVALID_ARG;
  const int pay = with_payload ? 1 : 0;
  for (int v = 0; v < 2; ++v) {
    if (seg_radix_tile(key_bytes_of(dtype), pay, v) == keys_per_tile) {
      ctx->seg_radix_variant[dtype][pay] = v;
      return AHS_OK;
    }
  }
  return ctx->fail(AHS_E_INVALID_ARG, "no radix tile of %u keys for this key type", keys_per_tile);
}
