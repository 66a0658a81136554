// Host level loop of the sample sort (general path, Sec. III-G.1).  Every
// table lives on the device; after each level the host reads back four
// counters (next segments, finished items, next tiles, overflow) to size the
// next launches.
#include <cstring>

#include "host_internal.hpp"
#include "samplesort.hpp"

namespace ahs {

namespace {

struct SsLayout {
  uint64_t seg_cap = 0, tile_cap = 0, item_cap = 0;
  size_t segA = 0, segB = 0, spl = 0, counts = 0, offs = 0, items = 0, ctr = 0, status = 0, tilectr = 0;
  size_t total = 0;
};

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

}  // namespace

size_t samplesort_ws_bytes(uint64_t n, int key_bytes, int) { return ss_layout(n, key_bytes).total; }

#define SS_HIP(call, what)                                  \
  do {                                                      \
    ahs_status st__ = j.ctx->check((call), (what));         \
    if (st__ != AHS_OK) return st__;                        \
  } while (0)

ahs_status run_samplesort(SortJob& j) {
  const SsLayout S = ss_layout(j.n, j.key_bytes);
  char* base = at<char>(j.ws, j.L.ss);
  SsSeg* segs[2] = {reinterpret_cast<SsSeg*>(base + S.segA), reinterpret_cast<SsSeg*>(base + S.segB)};
  void* spl = base + S.spl;
  uint32_t* counts = reinterpret_cast<uint32_t*>(base + S.counts);
  uint32_t* offs = reinterpret_cast<uint32_t*>(base + S.offs);
  SsItem* items = reinterpret_cast<SsItem*>(base + S.items);
  SsCounters* ctr = reinterpret_cast<SsCounters*>(base + S.ctr);
  void* status = base + S.status;
  const size_t sw = status_word_bytes(j.n);
  uint32_t* tilectr = reinterpret_cast<uint32_t*>(base + S.tilectr);
  const bool flt = j.kk == KK_F32 || j.kk == KK_F64;
  const int pay = j.vin != nullptr;

  SsBlockArgs ba;
  ba.items = items;
  ba.kin = j.kin;
  ba.kout = j.kout;
  ba.ktmp = at<void>(j.ws, j.L.tmpk);
  ba.vin = j.vin;
  ba.vout = j.vout;
  ba.vtmp = pay ? at<uint32_t>(j.ws, j.L.tmpv) : nullptr;

  SS_HIP(launch_ss_init(segs[0], items, j.n, j.s), "sample sort init");
  const double rec_bytes = 2.0 * j.key_bytes + (pay ? 8.0 : 0.0);  // read + write per key
  if (j.n <= (uint64_t)SS_CAP) {
    ProfScope p(j.ctx, "ss_block_sort", j.s, rec_bytes * j.n);
    SS_HIP(launch_ss_block(j.kk, pay, ba, 1, j.s), "block sort");
    return AHS_OK;
  }
  SS_HIP(launch_fill_u32(reinterpret_cast<uint32_t*>(ctr), sizeof(SsCounters) / 4 * SS_MAX_LEVELS, 0u, j.s), "fill");
  SS_HIP(launch_fill_u32(tilectr, SS_MAX_LEVELS, 0u, j.s), "fill");

  const void* bufs[3] = {j.kin, j.kout, at<void>(j.ws, j.L.tmpk)};
  const uint32_t* vbufs[3] = {j.vin, j.vout, ba.vtmp};
  const uint32_t tile_keys = (uint32_t)ss_tile(j.key_bytes);
  uint32_t nsegs = 1;
  uint32_t ntiles = (uint32_t)ceil_div(j.n, tile_keys);
  uint32_t src_buf = SS_BUF_IN;
  uint64_t level_keys = j.n;
  int cur = 0;
  for (int level = 0; level < SS_MAX_LEVELS; ++level) {
    const uint32_t dst_buf = (level % 2 == 0) ? SS_BUF_TMP : SS_BUF_OUT;
    const int map_in = (flt && src_buf == SS_BUF_IN) ? 1 : 0;
    SS_HIP(launch_fill_u32(counts, (uint64_t)nsegs * SS_NB, 0u, j.s), "fill");
    SS_HIP(launch_fill_u32(static_cast<uint32_t*>(status), (uint64_t)ntiles * SS_NB * sw / 4, 0u, j.s), "fill");
    {
      ProfScope p(j.ctx, "ss_sample", j.s);
      SS_HIP(launch_ss_sample(j.kk, bufs[src_buf], map_in, segs[cur], nsegs, spl, 0x5EEDull + (uint64_t)level, j.s),
             "sample");
    }
    {
      ProfScope p(j.ctx, "ss_count", j.s, (double)j.key_bytes * level_keys);
      const int nb = (int)(ntiles < 2048u ? ntiles : 2048u);
      SS_HIP(launch_ss_count(j.kk, bufs[src_buf], map_in, segs[cur], nsegs, ntiles, spl, counts, nb, j.s), "count");
    }
    SS_HIP(launch_ss_plan(segs[cur], nsegs, counts, offs, dst_buf, flt ? 1 : 0, segs[cur ^ 1], items, ctr + level,
                          (uint32_t)S.item_cap, (uint32_t)S.seg_cap, j.s),
           "plan");
    SsScatterArgs sa;
    sa.src = bufs[src_buf];
    sa.dst = const_cast<void*>(bufs[dst_buf]);
    sa.vsrc = pay ? vbufs[src_buf] : nullptr;
    sa.vdst = pay ? const_cast<uint32_t*>(vbufs[dst_buf]) : nullptr;
    sa.map_in = (uint32_t)map_in;
    sa.nsegs = nsegs;
    sa.segs = segs[cur];
    sa.spl = spl;
    sa.offs = offs;
    sa.status = status;
    sa.tile_counter = tilectr + level;
    sa.n = j.n;
    {
      ProfScope p(j.ctx, "ss_scatter", j.s, rec_bytes * level_keys);
      SS_HIP(launch_ss_scatter(j.kk, pay, sa, ntiles, j.s), "scatter");
    }
    SS_HIP(launch_ss_tiles(segs[cur ^ 1], ctr + level, tile_keys, (uint32_t)S.seg_cap, j.s), "tiles");
    SS_HIP(hipMemcpyAsync(j.ctx->pinned, ctr + level, sizeof(SsCounters), hipMemcpyDeviceToHost, j.s), "copy");
    SS_HIP(hipStreamSynchronize(j.s), "synchronize");
    SsCounters c;
    memcpy(&c, j.ctx->pinned, sizeof c);
    if (c.overflow) return j.ctx->fail(AHS_E_DEVICE, "sample sort table overflow (%u)", c.overflow);
    if (c.nitems) {
      ProfScope p(j.ctx, "ss_block_sort", j.s, rec_bytes * c.item_keys);
      SS_HIP(launch_ss_block(j.kk, pay, ba, c.nitems, j.s), "block sort");
    }
    if (c.nsegs_next == 0) return AHS_OK;
    nsegs = c.nsegs_next;
    ntiles = c.ntiles_next;
    level_keys = c.seg_keys_next;
    src_buf = dst_buf;
    cur ^= 1;
  }
  return j.ctx->fail(AHS_E_DEVICE, "sample sort did not converge in %d levels", SS_MAX_LEVELS);
}

}  // namespace ahs
