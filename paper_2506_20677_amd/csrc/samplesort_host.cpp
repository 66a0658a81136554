// Host level loops of the sample sort (general path, Sec. III-G.1).  Every
// table lives on the device.  The host-driven loop reads back one counter
// record per level (next segments, finished items, next tiles, overflow) to
// size the next launches exactly; the device-driven loop launches fixed
// grids whose kernels read those sizes themselves, so it never blocks.
#include <cmath>
#include <cstring>

#include "ss_host.hpp"

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
  L.spl = take(ss_spl_rec_bytes(key_bytes) * L.seg_cap);
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

namespace {

SsBlockArgs block_args(SortJob& j, const SsTables& T) {
  SsBlockArgs ba;
  ba.items = T.items;
  ba.lvl = nullptr;
  ba.nitems = 0;
  ba.item_cap = 0;
  ba.kin = j.kin;
  ba.kout = j.kout;
  ba.ktmp = at<void>(j.ws, j.L.tmpk);
  ba.vin = j.vin;
  ba.vout = j.vout;
  ba.vtmp = j.vin ? at<uint32_t>(j.ws, j.L.tmpv) : nullptr;
  return ba;
}

// Everything one level launches, given its sizes (host values, or the
// previous level's record when lv.in is set).
struct LevelPlan {
  int level;
  uint32_t src_buf, dst_buf;
  int cur;
  SsLevelIn lv;
  int sample_grid, count_grid, plan_grid;
  uint32_t scatter_grid;  // 0: one workgroup per tile
  double count_bytes, move_bytes;
};

ahs_status launch_level(SortJob& j, const SsLayout& S, const SsTables& T, const LevelPlan& P, uint64_t max_seg) {
  const bool mapped = j.kk == KK_F32 || j.kk == KK_F64 || j.kk == KK_I32 || j.kk == KK_I64;
  const int pay = j.vin != nullptr;
  const void* bufs[3] = {j.kin, j.kout, at<void>(j.ws, j.L.tmpk)};
  const uint32_t* vbufs[3] = {j.vin, j.vout, j.vin ? at<uint32_t>(j.ws, j.L.tmpv) : nullptr};
  const int map_in = (mapped && P.src_buf == SS_BUF_IN) ? 1 : 0;
  const uint32_t sw = (uint32_t)status_word_bytes(max_seg);
  {
    ProfScope p(j.ctx, "ss_sample", j.s);
    SS_HIP(launch_ss_sample(j.kk, bufs[P.src_buf], map_in, T.segs[P.cur], P.lv, T.spl, T.counts,
                            0x5EEDull + (uint64_t)P.level, P.sample_grid, j.s),
           "sample");
  }
  SS_HIP(launch_ss_zero_status(T.status, P.lv, SS_NB * sw / 4, j.s), "clear status");
  {
    ProfScope p(j.ctx, "ss_count", j.s, P.count_bytes);
    SS_HIP(launch_ss_count(j.kk, bufs[P.src_buf], map_in, T.segs[P.cur], P.lv, T.spl, T.counts, P.count_grid, j.s),
           "count");
  }
  // large buckets of equal keys go straight to the output unless it is
  // the level's source (an in-place call's level 0, or a level reading the
  // output)
  const bool eq_out = bufs[P.src_buf] != j.kout && (!pay || vbufs[P.src_buf] != j.vout);
  SS_HIP(launch_ss_plan(T.segs[P.cur], P.lv, T.counts, T.offs, P.dst_buf, mapped ? 1 : 0, eq_out ? 1 : 0, T.spl,
                        j.key_bytes, T.segs[P.cur ^ 1], T.items,
                        T.ctr + P.level, (uint32_t)S.item_cap, (uint32_t)S.seg_cap, P.plan_grid, j.s),
         "plan");
  SsScatterArgs sa;
  sa.src = bufs[P.src_buf];
  sa.dst = const_cast<void*>(bufs[P.dst_buf]);
  sa.vsrc = pay ? vbufs[P.src_buf] : nullptr;
  sa.vdst = pay ? const_cast<uint32_t*>(vbufs[P.dst_buf]) : nullptr;
  sa.map_in = (uint32_t)map_in;
  sa.lv = P.lv;
  sa.segs = T.segs[P.cur];
  sa.spl = T.spl;
  sa.offs = T.offs;
  sa.status = T.status;
  sa.tile_counter = T.tilectr + P.level;
  sa.max_seg = max_seg;
  sa.out = j.kout;
  sa.vout = pay ? j.vout : nullptr;
  {
    ProfScope p(j.ctx, "ss_scatter", j.s, P.move_bytes);
    SS_HIP(launch_ss_scatter(j.kk, pay, sa, P.scatter_grid, j.s), "scatter");
  }
  SS_HIP(launch_ss_tiles(T.segs[P.cur ^ 1], T.ctr + P.level, (uint32_t)ss_tile(j.key_bytes), (uint32_t)S.seg_cap,
                         j.s),
         "tiles");
  return AHS_OK;
}

// Levels a segment of max_seg keys is expected to take: splitters aim at
// SS_TARGET-key buckets (at most 255 per level), so a level takes a segment
// of up to 255 * SS_TARGET keys to single-level buckets and a larger one
// down by 256.
int expected_levels(uint64_t max_seg) {
  int e = 0;
  for (uint64_t s = max_seg; s > (uint64_t)SS_CAP; ++e)
    s = s <= (uint64_t)SS_P * SS_TARGET ? (uint64_t)SS_TARGET : ceil_div(s, (uint64_t)SS_P + 1);
  return e;
}

// Buffer a level scatters into.  The levels alternate between the scratch
// buffer and the output so that the last expected level writes the output:
// its buckets are then block-sorted in place there (sorting from the
// scratch buffer into the output measured 12 % slower).  An in-place call
// (output = input) starts in the scratch buffer, since level 0 reads the
// input.
uint32_t level_dst(const SortJob& j, int level, uint64_t max_seg) {
  const bool alias = j.kin == j.kout || (j.vin && j.vin == j.vout);
  const int last = expected_levels(max_seg) - 1;
  const bool out = alias ? (level % 2 == 1) : ((last - level) % 2 == 0);
  return out ? SS_BUF_OUT : SS_BUF_TMP;
}

ahs_status clear_counters(SortJob& j, const SsTables& T) {
  SS_HIP(launch_ss_init(nullptr, nullptr, 0, T.ctr, T.tilectr, SS_MAX_LEVELS, j.s), "clear counters");
  return AHS_OK;
}

}  // namespace

ahs_status ss_levels_host(SortJob& j, const SsLayout& S, const SsTables& T, uint32_t nsegs, uint32_t ntiles,
                          uint64_t level_keys, uint64_t max_seg, bool counters_cleared) {
  const int pay = j.vin != nullptr;
  const double rec_bytes = 2.0 * j.key_bytes + (pay ? 8.0 : 0.0);  // read + write per key
  SsBlockArgs ba = block_args(j, T);
  if (!counters_cleared) AHS_TRY(clear_counters(j, T));
  uint32_t src_buf = SS_BUF_IN;
  int cur = 0;
  for (int level = 0; level < SS_MAX_LEVELS; ++level) {
    if (nsegs == 0) return AHS_OK;
    LevelPlan P;
    P.level = level;
    P.src_buf = src_buf;
    P.dst_buf = level_dst(j, level, max_seg);
    P.cur = cur;
    P.lv = SsLevelIn{nullptr, nsegs, ntiles, (uint32_t)S.seg_cap, (uint32_t)S.tile_cap};
    P.sample_grid = (int)nsegs;
    P.count_grid = (int)(ntiles < 2048u ? ntiles : 2048u);
    P.plan_grid = (int)nsegs;
    P.scatter_grid = 0;
    P.count_bytes = (double)j.key_bytes * level_keys;
    P.move_bytes = rec_bytes * level_keys;
    AHS_TRY(launch_level(j, S, T, P, max_seg));
    SS_HIP(hipMemcpyAsync(j.ctx->pinned, T.ctr + level, sizeof(SsCounters), hipMemcpyDeviceToHost, j.s), "copy");
    SS_HIP(hipStreamSynchronize(j.s), "synchronize");
    SsCounters c;
    memcpy(&c, j.ctx->pinned, sizeof c);
    if (c.overflow) return j.ctx->fail(AHS_E_DEVICE, "sample sort table overflow (%u)", c.overflow);
    if (c.nitems) {
      ProfScope p(j.ctx, "ss_block_sort", j.s, rec_bytes * (double)c.item_keys);
      ba.nitems = c.nitems;
      SS_HIP(launch_ss_block(j.kk, pay, ba, 0, j.s), "block sort");
    }
    nsegs = c.nsegs_next;
    ntiles = c.ntiles_next;
    level_keys = c.seg_keys_next;
    src_buf = P.dst_buf;
    cur ^= 1;
  }
  if (nsegs == 0) return AHS_OK;
  return j.ctx->fail(AHS_E_DEVICE, "sample sort did not converge in %d levels", SS_MAX_LEVELS);
}

int ss_levels_for(uint64_t max_seg) {
  if (max_seg <= (uint64_t)SS_CAP) return 0;
  const int excess = bitlen64(max_seg - 1) - 13;  // log2 of max_seg / SS_CAP, rounded up
  return (excess + 5) / 6 + 1;
}

ahs_status ss_levels_device(SortJob& j, const SsLayout& S, const SsTables& T, const SsCounters* in0, int levels,
                            uint64_t max_seg) {
  const int pay = j.vin != nullptr;
  if (levels > SS_MAX_LEVELS) levels = SS_MAX_LEVELS;
  AHS_TRY(clear_counters(j, T));
  const uint32_t cu = j.ctx->cu_count ? j.ctx->cu_count : 256;
  const uint32_t seg_cap = (uint32_t)S.seg_cap;
  const int seg_grid = (int)(seg_cap < 2 * cu ? seg_cap : 2 * cu);
  const uint32_t scatter_grid = ss_scatter_resident(j.kk, pay, max_seg, cu);
  SsBlockArgs ba = block_args(j, T);
  ba.item_cap = (uint32_t)S.item_cap;
  const uint32_t block_grid = ss_block_resident(j.kk, pay, cu);
  uint32_t src_buf = SS_BUF_IN;
  int cur = 0;
  for (int level = 0; level < levels; ++level) {
    LevelPlan P;
    P.level = level;
    P.src_buf = src_buf;
    P.dst_buf = level_dst(j, level, max_seg);
    P.cur = cur;
    P.lv = SsLevelIn{level == 0 ? in0 : T.ctr + (level - 1), 0u, 0u, seg_cap, (uint32_t)S.tile_cap};
    P.sample_grid = seg_grid;
    P.count_grid = 2048;
    P.plan_grid = seg_grid;
    P.scatter_grid = scatter_grid;
    P.count_bytes = 0.0;  // sizes are known on the device only
    P.move_bytes = 0.0;
    AHS_TRY(launch_level(j, S, T, P, max_seg));
    ba.lvl = T.ctr + level;
    {
      ProfScope p(j.ctx, "ss_block_sort", j.s);
      SS_HIP(launch_ss_block(j.kk, pay, ba, block_grid, j.s), "block sort");
    }
    src_buf = P.dst_buf;
    cur ^= 1;
  }
  return AHS_OK;
}

ahs_status run_samplesort(SortJob& j) {
  const SsLayout S = ss_layout(j.n, j.key_bytes);
  const SsTables T = ss_tables(j, S);
  const int pay = j.vin != nullptr;
  // one launch: segment 0, item 0 and, when levels follow, their counters
  const bool levels = j.n > (uint64_t)SS_CAP;
  SS_HIP(launch_ss_init(T.segs[0], T.items, j.n, T.ctr, T.tilectr, levels ? SS_MAX_LEVELS : 0, j.s),
         "sample sort init");
  if (!levels) {
    ProfScope p(j.ctx, "ss_block_sort", j.s, (2.0 * j.key_bytes + (pay ? 8.0 : 0.0)) * j.n);
    SsBlockArgs ba = block_args(j, T);
    ba.nitems = 1;
    SS_HIP(launch_ss_block(j.kk, pay, ba, 0, j.s), "block sort");
    return AHS_OK;
  }
  return ss_levels_host(j, S, T, 1, (uint32_t)ceil_div(j.n, (uint64_t)ss_tile(j.key_bytes)), j.n, j.n, true);
}

}  // namespace ahs
