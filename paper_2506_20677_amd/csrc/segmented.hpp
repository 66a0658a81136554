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

struct SegConfig {  // the decision thresholds the device needs
  uint64_t n_small, k_count, k_radix;
  double h_ratio;
};

struct SegCounters {
  uint32_t nclass[SEG_NCLASS];
  uint32_t nlarge, bad, max_large, pad;
  unsigned long long large_keys, small_keys;
};

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

// Large segments go both to the sample sort's level-0 table (large_ss) and
// to a copy the feature kernel reads after the levels (large).
hipError_t launch_seg_classify(const uint64_t* offs, uint32_t nseg, uint64_t n_total, uint32_t* queues, uint32_t qcap,
                               SsSeg* large_ss, SsSeg* large, uint32_t* large_ids, SegCounters* ctr, hipStream_t s);
// Level-0 record of the sample sort and the chunk record: the large-segment
// count, or zero when the offsets were invalid.
hipError_t launch_seg_gate(const SegCounters* ctr, SsCounters* rec0, SsCounters* rec_chunks, hipStream_t s);
// Class `cls` through variant `variant` (capacity SEG_CLASS_CAP[variant] >=
// SEG_CLASS_CAP[cls]); the kernel reads the queue length from ctr.
hipError_t launch_seg_small(int kk, int with_vals, const SegArgs& a, int cls, int variant, uint32_t nblocks,
                            hipStream_t s);
// Features of the large segments after sorting: NaN bounds, per-chunk run
// entropy, then one workgroup per segment folds its chunks in order.
hipError_t launch_seg_large(int kk, const SegArgs& a, uint32_t bound_blocks, uint32_t chunk_blocks,
                            uint32_t final_blocks, hipStream_t s);
uint32_t seg_chunk_resident(int kk, uint32_t cu_count);
hipError_t launch_seg_status(const SegCounters* ctr, const SsCounters* levels, int nlevels, uint32_t* status,
                             hipStream_t s);
uint32_t seg_small_resident(int kk, int with_vals, int variant, uint32_t cu_count);
// Deterministic synthetic keys for the autotuner (a counter hash).
hipError_t launch_tune_fill(int kk, void* keys, uint64_t n, uint64_t seed, hipStream_t s);

}  // namespace ahs
