// Host-side pieces of the sample-sort level loop shared by the single-array
// general path and the batched segmented sort.
#pragma once

#include "host_internal.hpp"
#include "samplesort.hpp"

namespace ahs {

struct SsTables {
  SsSeg* segs[2];
  void* spl;
  uint32_t* counts;
  uint32_t* offs;
  SsItem* items;
  SsCounters* ctr;  // one record per level
  void* status;
  uint32_t* tilectr;
};

SsTables ss_tables(SortJob& j, const SsLayout& S);

// Host-driven levels over the nsegs segments in T.segs[0] (first_tile set,
// ntiles tiles, level_keys keys), level 0 reading the input buffer.  Reads
// one counter record per level back to size the next level's grids.
ahs_status ss_levels_host(SortJob& j, const SsLayout& S, const SsTables& T, uint32_t nsegs, uint32_t ntiles,
                          uint64_t level_keys, uint64_t max_seg,
                          bool counters_cleared = false);

// Device-driven levels: `levels` levels whose sizes the kernels read from
// the previous level's record (level 0 from *in0).  Never synchronises.
ahs_status ss_levels_device(SortJob& j, const SsLayout& S, const SsTables& T, const SsCounters* in0, int levels,
                            uint64_t max_seg);

// Levels a device-driven run launches for segments of at most max_seg keys:
// enough for a 64-fold shrink per level plus one.
int ss_levels_for(uint64_t max_seg);

}  // namespace ahs
