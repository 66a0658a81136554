// Sample-sort shapes, device tables and launchers shared by the kernels
// (samplesort.hip) and the host level loop (samplesort_host.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace ahs {

constexpr int SS_P = 255;             // splitters per segment
constexpr int SS_NB = 512;            // bucket-id space (2 * SS_P + 1 used)
constexpr int SS_SAMPLES = 8192;      // most sample keys per segment
constexpr int SS_CAP = 8192;          // largest bucket finished in LDS
constexpr int SS_TARGET = 4096;       // bucket size a level aims at (splitters per segment: size / SS_TARGET, <= 255)
constexpr int SS_THREADS = 512;
// Per-segment splitter record: the 255 splitters in ascending order and in
// search-tree order (256 slots each), the cell table of the bucket
// classification (cells + 1 counts as bytes, padded to words), the word
// holding the cell shift and the flags, and the plan's 512-bit mask of the
// buckets that go straight to the output.  64-bit keys take half the
// cells, which keeps three 64-bit scatter tiles per CU in LDS.
__host__ __device__ constexpr uint32_t ss_cells_log2(int key_bytes) { return key_bytes == 4 ? 10u : 9u; }
__host__ __device__ constexpr uint32_t ss_cell_words(int key_bytes) { return ((1u << ss_cells_log2(key_bytes)) + 4u) / 4u; }
__host__ __device__ constexpr size_t ss_word_offset(int key_bytes) {
  return (size_t)key_bytes * 512 + 4 * ss_cell_words(key_bytes);
}
__host__ __device__ constexpr size_t ss_eq_mask_offset(int key_bytes) { return ss_word_offset(key_bytes) + 4; }
__host__ __device__ constexpr size_t ss_spl_rec_bytes(int key_bytes) {
  return (ss_eq_mask_offset(key_bytes) + 64 + 15) / 16 * 16;
}
constexpr int SS_MAX_LEVELS = 48;
// u32 scatter tiles of 24 keys per thread measured 6 % faster than 16 on
// 2^28 keys; u64 keeps 8 (12 and 16 were slower).
#ifndef AHS_SS_IPT32
#define AHS_SS_IPT32 24
#endif
#ifndef AHS_SS_IPT64
#define AHS_SS_IPT64 8
#endif
constexpr int SS_IPT32 = AHS_SS_IPT32, SS_IPT64 = AHS_SS_IPT64;  // scatter keys per thread (tunable)
inline int ss_tile(int key_bytes) { return SS_THREADS * (key_bytes == 4 ? SS_IPT32 : SS_IPT64); }

constexpr uint32_t SS_BUF_IN = 0, SS_BUF_OUT = 1, SS_BUF_TMP = 2;
constexpr uint32_t SS_ITEM_COPY = 1;

struct SsSeg {        // a range of the current buffer still to be split
  uint64_t start;
  uint32_t size;
  uint32_t first_tile;
};
struct SsItem {       // a finished bucket: sort in LDS, or copy
  uint64_t start;
  uint32_t size;
  uint32_t flags;     // bit 0: copy only; bits 8..15: source buffer id
};
struct SsCounters {   // per level, written by the device, read by the host
  uint32_t nsegs_next, nitems, ntiles_next, overflow;
  unsigned long long item_keys, seg_keys_next;
};

// Segment holding tile `tile` (segments' first_tile ascend).
__device__ __forceinline__ uint32_t ss_seg_of_tile(const SsSeg* __restrict__ segs, uint32_t nsegs, uint32_t tile) {
  uint32_t lo = 0, hi = nsegs;  // largest s with first_tile <= tile
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (segs[mid].first_tile <= tile) lo = mid; else hi = mid;
  }
  return lo;
}

// Level sizes: the host passes them (host-driven levels), or a kernel reads
// them from the previous level's counter record `in` (device-driven levels,
// enqueue-only), clamped to the table capacities.
struct SsLevelIn {
  const SsCounters* in;  // null: use the host values
  uint32_t nsegs, ntiles;
  uint32_t seg_cap, tile_cap;
  __device__ __forceinline__ uint32_t segs_n() const {
    if (!in) return nsegs;
    const uint32_t v = in->nsegs_next;
    return v < seg_cap ? v : seg_cap;
  }
  __device__ __forceinline__ uint32_t tiles_n() const {
    if (!in) return ntiles;
    const uint32_t v = in->ntiles_next;
    return v < tile_cap ? v : tile_cap;
  }
};

struct SsScatterArgs {
  const void* src;
  void* dst;
  const uint32_t* vsrc;
  uint32_t* vdst;
  uint32_t map_in;
  SsLevelIn lv;
  const SsSeg* segs;
  const void* spl;
  const uint32_t* offs;
  void* status;        // [tiles][SS_NB] words of status_word_bytes(max_seg), zero before the launch
  uint32_t* tile_counter;
  uint64_t max_seg;    // largest segment (selects the status word size)
  // Final output: the buckets the plan marked in a segment's record (large
  // buckets of equal keys) are written there directly, unmapped and already
  // in place, instead of into dst.
  void* out;
  uint32_t* vout;
};

struct SsBlockArgs {
  const SsItem* items;
  const SsCounters* lvl;   // device item count (nitems), or null: host count
  uint32_t nitems, item_cap;
  const void* kin;
  void* kout;
  const void* ktmp;
  const uint32_t* vin;
  uint32_t* vout;
  const uint32_t* vtmp;
};

// Sample-sort scratch layout inside the workspace.
struct SsLayout {
  uint64_t seg_cap = 0, tile_cap = 0, item_cap = 0;
  size_t segA = 0, segB = 0, spl = 0, counts = 0, offs = 0, items = 0, ctr = 0, status = 0, tilectr = 0;
  size_t total = 0;
};
SsLayout ss_layout(uint64_t n, int key_bytes);

// Zeroes `levels` counter records and tile counters; with segs set, also
// makes [0, n) segment 0 and item 0.
hipError_t launch_ss_init(SsSeg* segs, SsItem* items, uint64_t n, SsCounters* ctr, uint32_t* tilectr, int levels,
                          hipStream_t s);
// Every level kernel loops over its work (segments, tiles, items) with a
// grid stride, so device-driven levels launch fixed grids.  The sample
// kernel also clears the level's bucket counts.
hipError_t launch_ss_sample(int kk, const void* src, int map_in, const SsSeg* segs, const SsLevelIn& lv, void* spl,
                            uint32_t* counts, uint64_t seed, int nblocks, hipStream_t s);
hipError_t launch_ss_zero_status(void* status, const SsLevelIn& lv, uint32_t words_per_tile, hipStream_t s);
hipError_t launch_ss_count(int kk, const void* src, int map_in, const SsSeg* segs, const SsLevelIn& lv,
                           const void* spl, uint32_t* counts, int nblocks, hipStream_t s);
// eq_out: large buckets of equal keys go straight to the output (marked in
// the segment's record for the scatter; no item); the host sets it when
// the output is not the level's source.
hipError_t launch_ss_plan(const SsSeg* segs, const SsLevelIn& lv, const uint32_t* counts, uint32_t* offs,
                          uint32_t dst_buf, int copy_in_place, int eq_out, void* spl, int key_bytes, SsSeg* next,
                          SsItem* items, SsCounters* ctr, uint32_t item_cap, uint32_t seg_cap, int nblocks,
                          hipStream_t s);
// The rule both the plan and the scatter apply: bucket b (odd ids hold keys
// equal to a splitter) of c keys goes straight to the output.
__host__ __device__ __forceinline__ bool ss_eq_to_out(uint32_t b, uint32_t c) {
  return (b & 1u) && c > (uint32_t)(SS_CAP / 2);
}
hipError_t launch_ss_tiles(SsSeg* segs, SsCounters* ctr, uint32_t tile_keys, uint32_t seg_cap, hipStream_t s);
// nblocks 0: one block per tile (host-driven); else a persistent grid.
hipError_t launch_ss_scatter(int kk, int with_vals, const SsScatterArgs& a, uint32_t nblocks, hipStream_t s);
hipError_t launch_ss_block(int kk, int with_vals, const SsBlockArgs& a, uint32_t nblocks, hipStream_t s);
// Resident workgroups of the scatter and block-sort kernels on the device.
uint32_t ss_scatter_resident(int kk, int with_vals, uint64_t max_seg, uint32_t cu_count);
uint32_t ss_block_resident(int kk, int with_vals, uint32_t cu_count);

}  // namespace ahs
