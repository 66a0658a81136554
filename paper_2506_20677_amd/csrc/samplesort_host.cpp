// Host level loop of the sample sort (general path, Sec. III-G.1) and the
// batched segmented sort built on it.  Every table lives on the device;
// after each level the host reads back one counter record (next segments,
// finished items, next tiles, overflow) to size the next launches.
#include <cmath>
#include <cstring>

#include "host_internal.hpp"
#include "samplesort.hpp"
#include "segmented.hpp"

namespace ahs {

SsLayout ss_layout(uint64_t n, int key_bytes) {
  SsLayout L;
  // segments of one level are disjoint and hold more than SS_CAP keys
  L.seg_cap = n / (SS_CAP + 1) + 1;
  L.tile_cap = ceil_div(n ? n : 1, (uint64_t)ss_tile(key_bytes)) + L.seg_cap;
  // per level: at most 511 buckets per segment plus the chunks of large
  // equal-key buckets
  L.item_cap = 511 * L.seg_cap + n / SS_CAP + 16;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.segA = take(sizeof(SsSeg) * L.seg_cap);
  L.segB = take(sizeof(SsSeg) * L.seg_cap);
  L.spl = take((size_t)key_bytes * 256 * L.seg_cap);
  L.counts = take(4 * (size_t)SS_NB * L.seg_cap);
  L.offs = take(4 * (size_t)SS_NB * L.seg_cap);
  L.items = take(sizeof(SsItem) * L.item_cap);
  L.ctr = take(sizeof(SsCounters) * SS_MAX_LEVELS);
  L.status = take(8 * (size_t)SS_NB * L.tile_cap);
  L.tilectr = take(4 * SS_MAX_LEVELS);
  L.total = o;
  return L;
}

size_t samplesort_ws_bytes(uint64_t n, int key_bytes, int) { return ss_layout(n, key_bytes).total; }

#define SS_HIP(call, what)                                  \
  do {                                                      \
    ahs_status st__ = j.ctx->check((call), (what));         \
    if (st__ != AHS_OK) return st__;                        \
  } while (0)

namespace {

struct SsTables {
  SsSeg* segs[2];
  void* spl;
  uint32_t* counts;
  uint32_t* offs;
  SsItem* items;
  SsCounters* ctr;
  void* status;
  uint32_t* tilectr;
};

SsTables ss_tables(SortJob& j, const SsLayout& S) {
  char* base = at<char>(j.ws, j.L.ss);
  SsTables T;
  T.segs[0] = reinterpret_cast<SsSeg*>(base + S.segA);
  T.segs[1] = reinterpret_cast<SsSeg*>(base + S.segB);
  T.spl = base + S.spl;
  T.counts = reinterpret_cast<uint32_t*>(base + S.counts);
  T.offs = reinterpret_cast<uint32_t*>(base + S.offs);
  T.items = reinterpret_cast<SsItem*>(base + S.items);
  T.ctr = reinterpret_cast<SsCounters*>(base + S.ctr);
  T.status = base + S.status;
  T.tilectr = reinterpret_cast<uint32_t*>(base + S.tilectr);
  return T;
}

SsBlockArgs block_args(SortJob& j, const SsTables& T) {
  SsBlockArgs ba;
  ba.items = T.items;
  ba.kin = j.kin;
  ba.kout = j.kout;
  ba.ktmp = at<void>(j.ws, j.L.tmpk);
  ba.vin = j.vin;
  ba.vout = j.vout;
  ba.vtmp = j.vin ? at<uint32_t>(j.ws, j.L.tmpv) : nullptr;
  return ba;
}

// Levels of the sample sort over the nsegs segments in T.segs[0] (their
// first_tile set, ntiles tiles in total, level_keys keys), reading level 0
// from the input buffer.  max_seg bounds every segment's size.
ahs_status ss_levels(SortJob& j, const SsLayout& S, const SsTables& T, uint32_t nsegs, uint32_t ntiles,
                     uint64_t level_keys, uint64_t max_seg) {
  const bool flt = j.kk == KK_F32 || j.kk == KK_F64;
  const int pay = j.vin != nullptr;
  const double rec_bytes = 2.0 * j.key_bytes + (pay ? 8.0 : 0.0);  // read + write per key
  const SsBlockArgs ba = block_args(j, T);
  SS_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(T.ctr), sizeof(SsCounters) / 4 * SS_MAX_LEVELS, 0u, j.s),
         "fill");
  SS_HIP(launch_fill_u32(T.tilectr, SS_MAX_LEVELS, 0u, j.s), "fill");
  const void* bufs[3] = {j.kin, j.kout, at<void>(j.ws, j.L.tmpk)};
  const uint32_t* vbufs[3] = {j.vin, j.vout, ba.vtmp};
  const uint32_t tile_keys = (uint32_t)ss_tile(j.key_bytes);
  const size_t sw = status_word_bytes(max_seg);
  uint32_t src_buf = SS_BUF_IN;
  int cur = 0;
  for (int level = 0; level < SS_MAX_LEVELS; ++level) {
    if (nsegs == 0) return AHS_OK;
    const uint32_t dst_buf = (level % 2 == 0) ? SS_BUF_TMP : SS_BUF_OUT;
    const int map_in = (flt && src_buf == SS_BUF_IN) ? 1 : 0;
    SS_HIP(launch_fill_u32(T.counts, (uint64_t)nsegs * SS_NB, 0u, j.s), "fill");
    SS_HIP(launch_fill_u32(static_cast<uint32_t*>(T.status), (uint64_t)ntiles * SS_NB * sw / 4, 0u, j.s), "fill");
    {
      ProfScope p(j.ctx, "ss_sample", j.s);
      SS_HIP(launch_ss_sample(j.kk, bufs[src_buf], map_in, T.segs[cur], nsegs, T.spl, 0x5EEDull + (uint64_t)level,
                              j.s),
             "sample");
    }
    {
      ProfScope p(j.ctx, "ss_count", j.s, (double)j.key_bytes * level_keys);
      const int nb = (int)(ntiles < 2048u ? ntiles : 2048u);
      SS_HIP(launch_ss_count(j.kk, bufs[src_buf], map_in, T.segs[cur], nsegs, ntiles, T.spl, T.counts, nb, j.s),
             "count");
    }
    SS_HIP(launch_ss_plan(T.segs[cur], nsegs, T.counts, T.offs, dst_buf, flt ? 1 : 0, T.segs[cur ^ 1], T.items,
                          T.ctr + level, (uint32_t)S.item_cap, (uint32_t)S.seg_cap, j.s),
           "plan");
    SsScatterArgs sa;
    sa.src = bufs[src_buf];
    sa.dst = const_cast<void*>(bufs[dst_buf]);
    sa.vsrc = pay ? vbufs[src_buf] : nullptr;
    sa.vdst = pay ? const_cast<uint32_t*>(vbufs[dst_buf]) : nullptr;
    sa.map_in = (uint32_t)map_in;
    sa.nsegs = nsegs;
    sa.segs = T.segs[cur];
    sa.spl = T.spl;
    sa.offs = T.offs;
    sa.status = T.status;
    sa.tile_counter = T.tilectr + level;
    sa.max_seg = max_seg;
    {
      ProfScope p(j.ctx, "ss_scatter", j.s, rec_bytes * level_keys);
      SS_HIP(launch_ss_scatter(j.kk, pay, sa, ntiles, j.s), "scatter");
    }
    SS_HIP(launch_ss_tiles(T.segs[cur ^ 1], T.ctr + level, tile_keys, (uint32_t)S.seg_cap, j.s), "tiles");
    SS_HIP(hipMemcpyAsync(j.ctx->pinned, T.ctr + level, sizeof(SsCounters), hipMemcpyDeviceToHost, j.s), "copy");
    SS_HIP(hipStreamSynchronize(j.s), "synchronize");
    SsCounters c;
    memcpy(&c, j.ctx->pinned, sizeof c);
    if (c.overflow) return j.ctx->fail(AHS_E_DEVICE, "sample sort table overflow (%u)", c.overflow);
    if (c.nitems) {
      ProfScope p(j.ctx, "ss_block_sort", j.s, rec_bytes * (double)c.item_keys);
      SS_HIP(launch_ss_block(j.kk, pay, ba, c.nitems, j.s), "block sort");
    }
    nsegs = c.nsegs_next;
    ntiles = c.ntiles_next;
    level_keys = c.seg_keys_next;
    src_buf = dst_buf;
    cur ^= 1;
  }
  if (nsegs == 0) return AHS_OK;
  return j.ctx->fail(AHS_E_DEVICE, "sample sort did not converge in %d levels", SS_MAX_LEVELS);
}

struct SegLayout {
  size_t thr = 0, small_ids = 0, large = 0, large_ids = 0, segctr = 0, total = 0;
};

SegLayout seg_layout(size_t base, uint32_t nseg) {
  SegLayout L;
  size_t o = base;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.thr = take(sizeof(double) * 65537);
  L.small_ids = take(4 * ((size_t)nseg + 1));
  L.large = take(sizeof(SsSeg) * ((size_t)nseg + 1));
  L.large_ids = take(4 * ((size_t)nseg + 1));
  L.segctr = take(sizeof(SegCounters) + sizeof(SsCounters));
  L.total = o;
  return L;
}

}  // namespace

ahs_status run_samplesort(SortJob& j) {
  const SsLayout S = ss_layout(j.n, j.key_bytes);
  const SsTables T = ss_tables(j, S);
  const int pay = j.vin != nullptr;
  SS_HIP(launch_ss_init(T.segs[0], T.items, j.n, j.s), "sample sort init");
  if (j.n <= (uint64_t)SS_CAP) {
    ProfScope p(j.ctx, "ss_block_sort", j.s, (2.0 * j.key_bytes + (pay ? 8.0 : 0.0)) * j.n);
    SS_HIP(launch_ss_block(j.kk, pay, block_args(j, T), 1, j.s), "block sort");
    return AHS_OK;
  }
  return ss_levels(j, S, T, 1, (uint32_t)ceil_div(j.n, (uint64_t)ss_tile(j.key_bytes)), j.n, j.n);
}

}  // namespace ahs

using namespace ahs;

extern "C" size_t ahs_segmented_workspace_bytes(uint64_t n_total, uint32_t nseg, ahs_dtype dtype, int with_payload) {
  if ((int)dtype < 0 || (int)dtype > 3) return 0;
  const int kb = (dtype == AHS_U32 || dtype == AHS_F32) ? 4 : 8;
  const Layout L = plan_layout(n_total, kb, with_payload ? 1 : 0, true);
  return seg_layout(L.total, nseg).total;
}

extern "C" ahs_status ahs_sort_segmented(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                                         const uint32_t* d_vals_in, uint32_t* d_vals_out, const uint64_t* d_offsets,
                                         uint32_t nseg, uint64_t n_total, ahs_dtype dtype, ahs_strategy requested,
                                         const ahs_config* cfg, void* d_ws, size_t ws_bytes, void* stream,
                                         uint8_t* d_chosen, ahs_feature_vector* d_feats) {
  if (!ctx) return AHS_E_INVALID_ARG;
  if ((int)dtype < 0 || (int)dtype > 3) return ctx->fail(AHS_E_INVALID_ARG, "bad dtype");
  if ((int)requested < AHS_AUTO || (int)requested > AHS_QUICK)
    return ctx->fail(AHS_E_INVALID_ARG, "strategy %d cannot be requested", (int)requested);
  if ((d_vals_in == nullptr) != (d_vals_out == nullptr))
    return ctx->fail(AHS_E_INVALID_ARG, "payload pointers must be both null or both set");
  ahs_config c;
  if (cfg) c = *cfg; else ahs_config_init(&c, AHS_PRESET_GPU);
  if (c.use_model) return ctx->fail(AHS_E_UNSUPPORTED, "the batched sort does not evaluate the model");
  if (c.k_count == 0) return ctx->fail(AHS_E_INVALID_ARG, "k_count must be positive");
  if (nseg == 0) return AHS_OK;
  if (!d_offsets || !d_ws || (n_total && (!d_keys_in || !d_keys_out)))
    return ctx->fail(AHS_E_INVALID_ARG, "null device pointer");
  const int kb = (dtype == AHS_U32 || dtype == AHS_F32) ? 4 : 8;
  if (d_keys_in != d_keys_out) {
    const uintptr_t x = (uintptr_t)d_keys_in, y = (uintptr_t)d_keys_out;
    if (x < y + kb * n_total && y < x + kb * n_total)
      return ctx->fail(AHS_E_INVALID_ARG, "input and output partially overlap");
  }

  SortJob j;
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
  const SegLayout G = seg_layout(j.L.total, nseg);
  if (ws_bytes < G.total) return ctx->fail(AHS_E_WORKSPACE, "workspace %zu < %zu", ws_bytes, G.total);
  SS_HIP(hipSetDevice(ctx->device), "set device");

  // threshold table, computed with the host's log2 exactly as ahs_select does
  double* thr_h = reinterpret_cast<double*>(static_cast<char*>(ctx->pinned) + (256 << 10));
  thr_h[0] = 0.0;
  for (uint32_t b = 1; b <= 65536; ++b) thr_h[b] = c.h_ratio * std::log2((double)b);
  double* thr = at<double>(d_ws, G.thr);
  SS_HIP(hipMemcpyAsync(thr, thr_h, sizeof(double) * 65537, hipMemcpyHostToDevice, j.s), "copy thresholds");

  const SsLayout S = ss_layout(n_total, kb);
  const SsTables T = ss_tables(j, S);
  SegCounters* sctr = at<SegCounters>(d_ws, G.segctr);
  SsCounters* tctr = reinterpret_cast<SsCounters*>(sctr + 1);
  uint32_t* small_ids = at<uint32_t>(d_ws, G.small_ids);
  SsSeg* large = at<SsSeg>(d_ws, G.large);
  uint32_t* large_ids = at<uint32_t>(d_ws, G.large_ids);
  SS_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(sctr), (sizeof(SegCounters) + sizeof(SsCounters)) / 4, 0u, j.s),
         "fill");
  {
    ProfScope p(ctx, "seg_classify", j.s);
    SS_HIP(launch_seg_classify(d_offsets, nseg, n_total, small_ids, T.segs[0], large, large_ids, sctr, j.s),
           "classify");
  }
  // tile numbering of the large segments (level 0 of the sample sort)
  SS_HIP(hipMemcpyAsync(&tctr->nsegs_next, &sctr->nlarge, 4, hipMemcpyDeviceToDevice, j.s), "copy");
  SS_HIP(launch_ss_tiles(T.segs[0], tctr, (uint32_t)ss_tile(kb), (uint32_t)S.seg_cap, j.s), "tiles");
  char* pin = static_cast<char*>(ctx->pinned);
  SS_HIP(hipMemcpyAsync(pin, sctr, sizeof(SegCounters) + sizeof(SsCounters), hipMemcpyDeviceToHost, j.s), "copy");
  SS_HIP(hipStreamSynchronize(j.s), "synchronize");
  SegCounters sc;
  SsCounters tc;
  memcpy(&sc, pin, sizeof sc);
  memcpy(&tc, pin + sizeof sc, sizeof tc);
  if (sc.bad) return ctx->fail(AHS_E_INVALID_ARG, "offsets are not non-decreasing or do not end at n_total");

  SegArgs a;
  a.kin = d_keys_in;
  a.kout = d_keys_out;
  a.vin = d_vals_in;
  a.vout = d_vals_out;
  a.offs = d_offsets;
  a.small_ids = small_ids;
  a.large = large;
  a.large_ids = large_ids;
  a.thr = thr;
  a.cfg.n_small = c.n_small;
  a.cfg.k_count = c.k_count;
  a.cfg.k_radix = c.k_radix;
  a.requested = (uint32_t)requested;
  a.chosen = d_chosen;
  a.feats = reinterpret_cast<DevFeatures*>(d_feats);
  const double rec_bytes = 2.0 * kb + (d_vals_in ? 8.0 : 0.0);
  {
    ProfScope p(ctx, "seg_small", j.s, rec_bytes * (double)(n_total - sc.large_keys));
    SS_HIP(launch_seg_small(j.kk, d_vals_in != nullptr, a, sc.nsmall, j.s), "small segments");
  }
  if (sc.nlarge) {
    ahs_status st = ss_levels(j, S, T, sc.nlarge, tc.ntiles_next, sc.large_keys, sc.max_large);
    if (st != AHS_OK) return st;
    ProfScope p(ctx, "seg_large_features", j.s, (double)kb * (double)sc.large_keys);
    SS_HIP(launch_seg_large(j.kk, a, sc.nlarge, j.s), "large-segment features");
  }
  return AHS_OK;
}
