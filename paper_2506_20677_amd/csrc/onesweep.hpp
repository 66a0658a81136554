// Tile-level building blocks of the single-pass ("onesweep") stable digit
// scatter on gfx950, shared by the LSD radix passes and the sample-sort
// bucket scatter.
//
// A tile of OS_THREADS * IPT keys is ranked stably by an 8-bit digit:
//   1. wave-level peer discovery without ballot chains: every lane ORs its
//      lane bit into an LDS mask slot indexed by its digit (ds_or_b64, order
//      irrelevant) and reads the slot back, which yields exactly the lanes
//      sharing its digit; the group leader (highest lane) clears the slot.
//      A wave whose 64 keys share one digit takes a ballot fast path.
//   2. each wave keeps running per-digit counts over its IPT items, so the
//      rank of a key inside its wave is (earlier items) + (lower lanes);
//   3. an exclusive scan over waves per digit gives wave prefixes, a scan
//      over digits gives tile-local digit starts.
// Key order inside a tile is (wave, item, lane), i.e. increasing index, so
// the ranks are stable.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace ahs {

template <int IPT>
__device__ __forceinline__ void rank_wave_items(const uint32_t (&d)[IPT], uint32_t (&r)[IPT],
                                                uint64_t* __restrict__ wmask /* [256] of this wave */,
                                                uint32_t* __restrict__ whist /* [256] of this wave */) {
  const int lane = lane_id();
  const uint64_t mybit = 1ull << lane;
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint32_t di = d[i];
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(di);
    const uint64_t same = __ballot(di == d0);
    uint64_t peers;
    const bool uniform = (same == ~0ull);
    if (uniform) {
      peers = ~0ull;
    } else {
      __hip_atomic_fetch_or(&wmask[di], mybit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __builtin_amdgcn_wave_barrier();
      peers = __hip_atomic_load(&wmask[di], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __builtin_amdgcn_wave_barrier();
    }
    const uint32_t lt = mbcnt(peers);
    const uint32_t cnt = popc64(peers);
    const uint32_t base = whist[di];
    __builtin_amdgcn_wave_barrier();
    r[i] = base + lt;
    if (lt == cnt - 1) {
      whist[di] = base + cnt;
      if (!uniform) wmask[di] = 0ull;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// After rank_wave_items on every wave and a __syncthreads: threads t < ND
// turn the per-wave counts of digit t into per-wave exclusive prefixes
// (in place) and return the tile's count of digit t (0 for t >= ND).
template <int NW, int ND = 256>
__device__ __forceinline__ uint32_t wave_prefix_per_digit(uint32_t (*whist)[ND]) {
  const int t = threadIdx.x;
  uint32_t run = 0;
  if (t < ND) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint32_t c = whist[w][t];
      whist[w][t] = run;
      run += c;
    }
  }
  return run;
}

// Decoupled look-back over tiles for digit t (called by threads t < ND).
// Publishes the tile aggregate, walks back to the nearest inclusive prefix
// and publishes the tile's own inclusive prefix.  Returns the exclusive
// prefix of this tile for digit t.  The chain starts at first_tile (the
// first tile of the tile's segment).  Tiles are numbered in launch order
// from an atomic counter, so every predecessor is resident and progresses.
template <int ND = 256>
__device__ __forceinline__ uint64_t lookback(uint64_t* __restrict__ status, uint32_t tile, uint32_t first_tile,
                                             uint32_t t, uint64_t count, uint32_t epoch) {
  const uint64_t ep = (uint64_t)epoch << ST_EPOCH_SHIFT;
  uint64_t* mine = status + (uint64_t)tile * ND + t;
  if (tile == first_tile) {
    st_agent(mine, ST_INC | ep | count);
    return 0;
  }
  st_agent(mine, ST_AGG | ep | count);
  uint64_t excl = 0;
  int64_t j = (int64_t)tile - 1;
  for (;;) {
    const uint64_t s = ld_agent(status + (uint64_t)j * ND + t);
    const uint64_t flag = s & ST_FLAG_MASK;
    if (flag == 0 || ((s >> ST_EPOCH_SHIFT) & 63u) != epoch) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += s & ST_VALUE_MASK;
    if (flag == ST_INC) break;
    --j;
  }
  st_agent(mine, ST_INC | ep | (excl + count));
  return excl;
}

}  // namespace ahs
