// Batched segmented sort: device tables and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"
#include "samplesort.hpp"

namespace ahs {

constexpr uint8_t SEG_STATUS_NAN = 0xFD;  // per-segment status: the segment holds NaN keys

struct SegConfig {  // the decision thresholds the device needs
  uint64_t n_small, k_count, k_radix;
};

struct SegCounters {
  uint32_t nsmall, nlarge, bad, max_large;
  unsigned long long large_keys, pad;
};

struct SegArgs {
  const void* kin;
  void* kout;
  const uint32_t* vin;
  uint32_t* vout;
  const uint64_t* offs;
  const uint32_t* small_ids;
  const SsSeg* large;
  const uint32_t* large_ids;
  const double* thr;        // thr[B] = h_ratio * log2(B), B = 0..65536
  SegConfig cfg;
  uint32_t requested;       // 0 = AUTO, else the forced strategy reported for every segment
  uint8_t* chosen;          // [nseg] or null
  DevFeatures* feats;       // [nseg] or null
};

hipError_t launch_seg_classify(const uint64_t* offs, uint32_t nseg, uint64_t n_total, uint32_t* small_ids, SsSeg* large,
                               SsSeg* large_copy, uint32_t* large_ids, SegCounters* ctr, hipStream_t s);
hipError_t launch_seg_small(int kk, int with_vals, const SegArgs& a, uint32_t nsmall, hipStream_t s);
hipError_t launch_seg_large(int kk, const SegArgs& a, uint32_t nlarge, hipStream_t s);

}  // namespace ahs
