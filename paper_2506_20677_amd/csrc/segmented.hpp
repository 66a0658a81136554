// Batched segmented sort: device tables and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "samplesort.hpp"

namespace ahs {

constexpr uint8_t SEG_STATUS_NAN = 0xFD;  // per-segment status: the segment holds NaN keys

// Small segments (at most SS_CAP keys) are queued by size class; class c
// holds sizes in (SEG_CLASS_CAP[c-1], SEG_CLASS_CAP[c]].  Each class runs one
// of the fused LDS kernel variants whose capacity covers it.
constexpr int SEG_NCLASS = 4;
constexpr uint32_t SEG_CLASS_CAP[SEG_NCLASS] = {1024, 2048, 4096, 8192};
constexpr int SEG_NVARIANT = 4;  // variant v has capacity SEG_CLASS_CAP[v]

// Device status word of the enqueue-only form.
constexpr uint32_t SEG_ERR_OFFSETS = 1u;   // offsets not non-decreasing, past n_total or a segment >= 2^32
constexpr uint32_t SEG_ERR_OVERFLOW = 2u;  // sample-sort table overflow
constexpr uint32_t SEG_ERR_LEVELS = 4u;    // a large segment still unsplit after the launched levels
constexpr uint32_t SEG_ERR_HINT = 8u;      // a segment larger than max_seg_hint

struct SegConfig {  // the decision thresholds the device needs
  uint64_t n_small, k_count, k_radix;
  double h_ratio;
};

// Decision engine of Sec. III-A on the device: n, then k = span + 1, then
// the entropy test against h_ratio * log2(B).
__device__ __forceinline__ uint8_t seg_fsm(uint64_t n, uint64_t span, uint32_t nbins, double H, const SegConfig& c) {
  if (n <= c.n_small) return 4;                                             // INSERTION
  if (span <= c.k_count - 1) return 1;                                      // COUNTING
  if (span >= c.k_radix && H < c.h_ratio * log2((double)nbins)) return 2;  // RADIX
  return 3;                                                                 // QUICK
}

// Bin shift and bin count of a span (at most 65,536 bins).
__device__ __forceinline__ void shift_nbins(uint64_t span, uint32_t& shift, uint32_t& nbins) {
  const int bl = bitlen64(span);
  shift = bl > 16 ? (uint32_t)(bl - 16) : 0u;
  nbins = (uint32_t)(span >> shift) + 1u;
}

struct SegCounters {
  uint32_t nclass[SEG_NCLASS];
  uint32_t nlarge, bad, max_large, pad;
  unsigned long long large_keys, small_keys;
};

// ------------------------------------------------------------------ large-segment dispatch
// Every large segment gets its features and its decision (Sec. III-A)
// before it is sorted, and the decision picks the kernel family that sorts
// it: COUNTING and RADIX segments go through segmented LSD passes over
// 8-bit digits of key - min (a counting sort over at most 2^16 values is the
// same stable scatter by the bin index, in one or two digit passes), QUICK
// segments through the sample-sort levels.  Min/max come from a chunked
// pass over all large segments; the entropy, needed only where the span
// reaches k_radix, from LDS histograms: one unit (workgroup) for a segment
// of at most SEG_HU keys, units of SEG_HU_MULTI keys for a larger one (whose
// units add into one global histogram per segment), so that one large
// segment alone still spreads over many CUs.
constexpr uint32_t SEG_HU = 1u << 20;            // largest single-unit segment
constexpr uint32_t SEG_HU_MULTI = 1u << 18;      // unit of a larger segment
__host__ __device__ __forceinline__ uint32_t seg_hist_unit_keys(uint32_t size) {
  return size <= SEG_HU ? SEG_HU : SEG_HU_MULTI;
}
constexpr int SEG_HIST_THREADS = 1024;
constexpr int SEG_HIST_EVENTS = 2 * (SEG_HU / 65536);  // bin corrections a unit can need
constexpr int SEG_MAX_PASSES = 9;                // 8 digits, plus a repeated first pass (in place)
constexpr int SEG_RD_THREADS = 512;              // radix pass and digit-count workgroups

struct SegLarge {                  // per large segment (index into the large list)
  unsigned long long mn, mx;       // min / max of the mapped non-NaN keys
  uint32_t nan;                    // NaN keys
  uint32_t pad;
};
struct SegRadixInfo {              // per segment of the radix list
  uint64_t kmin;
  uint32_t large;                  // index into the large list
  uint32_t ndig;                   // 8-bit digits of its span
  uint32_t npass;                  // digit passes (planned on the device)
  uint8_t pass[SEG_MAX_PASSES];    // digit of each pass, LSD order
  uint8_t pad[3];
};
struct SegDispatchCounters {
  SsCounters hist;                 // hist list (nsegs_next) and its units (ntiles_next)
  SsCounters radix;                // radix list (nsegs_next) and its tiles (ntiles_next)
  uint32_t tile_ctr[SEG_MAX_PASSES + 1];  // tile counters: digit count, then each pass
  uint32_t max_npass;
  uint32_t nslot;                  // global histograms of multi-unit segments in use
  uint32_t bad;                    // a capacity was exceeded (bit 1 of the status word)
};

struct SegDispatchArgs {
  const void* kin;
  void* kout;
  void* ktmp;
  const uint32_t* vin;
  uint32_t* vout;
  uint32_t* vtmp;
  const SsSeg* large;              // the large list (first_tile: first SEG_CH chunk)
  const uint32_t* large_ids;
  const SegCounters* ctr;
  const SsCounters* chunks;        // large-list chunks (ntiles_next)
  uint32_t chunk_cap;
  SegLarge* linfo;                 // [list_cap]
  SsSeg* qsegs;                    // sample-sort level 0 (the quick list)
  SsCounters* qrec;
  uint32_t qcap;
  SsSeg* hsegs;                    // hist list (first_tile: first unit)
  uint32_t* hlarge;                // its large-list indices
  uint32_t* hslots;                // [slot_cap][65,536] histograms of multi-unit segments
  uint32_t* hslot_of;              // [list_cap] slot of each hist-list segment (multi-unit only)
  uint32_t slot_cap;
  SsSeg* rsegs;                    // radix list (first_tile: first tile)
  SegRadixInfo* rinfo;
  uint32_t* rdig;                  // [list_cap][8][256] digit counts, then segment-relative offsets
  uint32_t list_cap;
  uint32_t tile_cap;               // radix tiles
  uint32_t unit_cap;               // hist units
  SegDispatchCounters* dctr;
  void* status;                    // look-back words of the radix passes
  SegConfig cfg;
  uint32_t requested;
  uint32_t in_place;               // keys or payload sorted in place
  uint8_t* chosen;
};

// Large-segment min/max and NaN counts (chunked), the decisions that need no
// entropy, the hist-list entropies and decisions, then the radix list's
// digit counts and pass plans.  Every kernel reads its counts from the
// device.  The quick list goes to qsegs/qrec (tiles still to be numbered).
hipError_t launch_seg_dispatch(int kk, const SegDispatchArgs& a, uint32_t cu_count, hipStream_t s);
// Numbers the radix tiles (tile_keys keys each) and counts the digits.
hipError_t launch_seg_radix_prepare(int kk, const SegDispatchArgs& a, uint32_t tile_keys, uint32_t cu_count,
                                    hipStream_t s);
// Pass q of the segmented LSD radix (q < SEG_MAX_PASSES); ipt_variant 0
// or 1 picks the tile size (seg_radix_tile).
hipError_t launch_seg_radix_pass(int kk, int with_vals, int ipt_variant, const SegDispatchArgs& a, int q,
                                 uint64_t max_seg, uint32_t cu_count, hipStream_t s);
uint32_t seg_radix_tile(int key_bytes, int with_vals, int ipt_variant);

// Features of large segments are taken from their sorted output in chunks
// of SEG_CH keys spread over the whole grid.
constexpr uint32_t SEG_CH = 8192;
constexpr int SEG_CH_THREADS = 256;

struct SegArgs {
  const void* kin;
  void* kout;
  const uint32_t* vin;
  uint32_t* vout;
  const uint64_t* offs;
  const uint32_t* queues;   // [SEG_NCLASS][qcap] small segment ids by class
  uint32_t qcap;
  const SsSeg* large;       // [nlarge] large segments (sample-sort level 0)
  const uint32_t* large_ids;
  const SegCounters* ctr;
  const SsCounters* chunks;  // nsegs_next = large segments, ntiles_next = their chunks (first chunk in large[].first_tile)
  uint32_t chunk_cap;
  uint32_t* bounds;          // [2 * nlarge]: first and end index of the non-NaN keys of each sorted large segment
  double* partial;           // [chunk_cap] entropy terms of the runs that end in each chunk
  SegConfig cfg;
  uint32_t requested;       // 0 = AUTO, else the forced strategy reported for every segment
  uint8_t* chosen;          // [nseg] or null
  DevFeatures* feats;       // [nseg] or null
};

// Large segments go to the large list (with a cleared min/max record each);
// the dispatch kernels decide and sort them.
hipError_t launch_seg_classify(const uint64_t* offs, uint32_t nseg, uint64_t n_total, uint32_t* queues, uint32_t qcap,
                               SegLarge* linfo, SsSeg* large, uint32_t* large_ids, SegCounters* ctr, hipStream_t s);
// The chunk record of the large list: its segment count, or zero when the
// offsets were invalid.
hipError_t launch_seg_gate(const SegCounters* ctr, SsCounters* rec_chunks, hipStream_t s);
// Class `cls` through variant `variant` (capacity SEG_CLASS_CAP[variant] >=
// SEG_CLASS_CAP[cls]); the kernel reads the queue length from ctr.
hipError_t launch_seg_small(int kk, int with_vals, const SegArgs& a, int cls, int variant, uint32_t nblocks,
                            hipStream_t s);
// Features of the large segments after sorting: NaN bounds, per-chunk run
// entropy, then one workgroup per segment folds its chunks in order.
hipError_t launch_seg_large(int kk, const SegArgs& a, uint32_t bound_blocks, uint32_t chunk_blocks,
                            uint32_t final_blocks, hipStream_t s);
uint32_t seg_chunk_resident(int kk, uint32_t cu_count);
hipError_t launch_seg_status(const SegCounters* ctr, const SsCounters* levels, int nlevels,
                             const SegDispatchCounters* dctr, uint64_t max_seg, uint32_t* status, hipStream_t s);
uint32_t seg_small_resident(int kk, int with_vals, int variant, uint32_t cu_count);
// Deterministic synthetic keys for the autotuner (a counter hash).
hipError_t launch_tune_fill(int kk, void* keys, uint64_t n, uint64_t seed, hipStream_t s);

}  // namespace ahs
