// Tile-level building blocks of the single-pass ("onesweep") stable digit
// scatter on gfx950, shared by the LSD radix passes and the sample-sort
// bucket scatter.
//
// A tile of OS_THREADS * IPT keys is ranked stably by an 8-bit digit:
//   1. wave-level peer discovery without ballot chains: every lane ORs its
//      lane bit into an LDS mask word indexed by its digit (ds_or_b64, order
//      irrelevant) and reads the word back, which yields exactly the lanes
//      sharing its digit; the group leader (highest lane) clears the word.
//      A wave whose 64 keys share one digit takes a ballot fast path.
//   2. each wave keeps running per-digit counts over its IPT items, so the
//      rank of a key inside its wave is (earlier items) + (lower lanes);
//   3. an exclusive scan over waves per digit gives wave prefixes, a scan
//      over digits gives tile-local digit starts; their sums go into a
//      dense per-(wave, digit) table of tile positions laid over the slots,
//      so each key's position costs one LDS read.
// Key order inside a tile is (wave, item, lane), i.e. increasing index, so
// the ranks are stable.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace ahs {

// Rank state of one wave over ND digits: the peer mask of the item being
// ranked and the wave's running count of each digit, kept in two arrays.
// Their 8- and 4-byte strides spread a wave's 64 random digits over more
// LDS banks than one 16-byte slot per digit did (that layout cost about a
// third more time in the ranking of a 2^28-key pass).
template <int ND>
struct RankLds {
  uint64_t mask[ND];
  uint32_t count[ND];
};
typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// Zeroes the rank state of `nw` waves (the whole workgroup of NT threads
// takes part; no barrier).
template <int ND, int NT>
__device__ __forceinline__ void rank_clear(RankLds<ND>* st, int nw) {
  static_assert(sizeof(RankLds<ND>) % 16 == 0, "rank state clears as 16-byte words");
  u32x4* p = reinterpret_cast<u32x4*>(st);
  const int nvec = nw * (int)(sizeof(RankLds<ND>) / 16);
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (int i = (int)threadIdx.x; i < nvec; i += NT) p[i] = z;
}

// Ranks items [0, nitems) of the wave (nitems wave-uniform; later items
// are left unranked and must not be used).  `st` lives in LDS.
template <int IPT, int ND>
__device__ __forceinline__ void rank_wave_items(const uint32_t (&d)[IPT], uint32_t (&r)[IPT], RankLds<ND>& st,
                                                int nitems = IPT) {
  lds_u64* mask = (lds_u64*)st.mask;
  lds_u32* count = (lds_u32*)st.count;
  const int lane = lane_id();
  const uint64_t mybit = 1ull << lane;
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    if (i < nitems) {  // uniform branch; the loop stays unrolled (static register indexing)
      const uint32_t di = d[i];
      const uint32_t d0 = __builtin_amdgcn_readfirstlane(di);
      if (__ballot(di == d0) == ~0ull) {
        // the whole wave shares one digit
        const uint32_t base = count[d0];
        __builtin_amdgcn_wave_barrier();
        r[i] = base + (uint32_t)lane;
        if (lane == WAVE - 1) count[d0] = base + WAVE;
      } else {
        __hip_atomic_fetch_or(&mask[di], mybit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __builtin_amdgcn_wave_barrier();
        const uint64_t peers = *(const volatile lds_u64*)&mask[di];
        const uint32_t base = *(const volatile lds_u32*)&count[di];
        __builtin_amdgcn_wave_barrier();
        const uint32_t lt = mbcnt(peers);
        const uint32_t cnt = popc64(peers);
        r[i] = base + lt;
        if (lt == cnt - 1) {
          *(volatile lds_u64*)&mask[di] = 0ull;
          *(volatile lds_u32*)&count[di] = base + cnt;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// Look-back status words.  32-bit words (flag in bits 31..30, value in
// 29..0) serve every array below 2^30 keys and halve the look-back traffic;
// 64-bit words (flag 63..62, value 55..0) serve the rest.  Status arrays are
// cleared before every pass, so a zero flag means "not published".
template <typename ST> struct Status;
template <> struct Status<uint32_t> {
  static constexpr uint32_t AGG = 1u << 30, INC = 2u << 30, FLAGS = 3u << 30, VAL = (1u << 30) - 1;
};
template <> struct Status<uint64_t> {
  static constexpr uint64_t AGG = 1ull << 62, INC = 2ull << 62, FLAGS = 3ull << 62, VAL = (1ull << 56) - 1;
};

// Decoupled look-back over tiles for digit t (called by threads t < ND).
// Publishes the tile aggregate, walks back to the nearest inclusive prefix
// and publishes the tile's own inclusive prefix.  Returns the exclusive
// prefix of this tile for digit t.  The chain starts at first_tile (the
// first tile of the tile's segment).  Tiles are numbered in launch order
// from an atomic counter, so every predecessor is resident and progresses.
//
// The walk first reads the direct predecessor alone (usually enough once
// the pass is running); if that one only holds an aggregate it reads the
// next LB_WIDTH predecessors with independent loads per round, so the
// inclusive frontier is not limited to one tile per load latency.
#ifndef AHS_LB_WIDTH
#define AHS_LB_WIDTH 4
#endif
#ifndef AHS_LB_SLEEP
#define AHS_LB_SLEEP 1
#endif
constexpr int LB_WIDTH = AHS_LB_WIDTH;  // predecessors read per round of the walk (compile-time tunable)

__device__ __forceinline__ void lb_pause() {
  if constexpr (AHS_LB_SLEEP > 0) __builtin_amdgcn_s_sleep(AHS_LB_SLEEP);
}

template <int ND, typename ST>
__device__ __forceinline__ uint64_t lookback(ST* __restrict__ status, uint32_t tile, uint32_t first_tile,
                                             uint32_t t, uint64_t count) {
  using S = Status<ST>;
  ST* mine = status + (uint64_t)tile * ND + t;
  if (tile == first_tile) {
    st_agent(mine, (ST)(S::INC | (ST)count));
    return 0;
  }
  st_agent(mine, (ST)(S::AGG | (ST)count));
  uint64_t excl = 0;
  int64_t j = (int64_t)tile - 1;  // next predecessor not yet accounted for
  // direct predecessor
  for (;;) {
    const ST s = ld_agent(status + (uint64_t)j * ND + t);
    if ((s & S::FLAGS) == 0) {
      lb_pause();
      continue;
    }
    excl += s & S::VAL;
    if ((s & S::FLAGS) == S::INC) {
      st_agent(mine, (ST)(S::INC | (ST)(excl + count)));
      return excl;
    }
    --j;
    break;
  }
  for (;;) {
    ST s[LB_WIDTH];
#pragma unroll
    for (int q = 0; q < LB_WIDTH; ++q)
      s[q] = (j - q >= (int64_t)first_tile) ? ld_agent(status + (uint64_t)(j - q) * ND + t) : (ST)0;
    int q = 0;
    bool done = false;
    for (; q < LB_WIDTH && j - q >= (int64_t)first_tile; ++q) {
      const ST flag = s[q] & S::FLAGS;
      if (flag == 0) break;  // not published yet: re-read from here
      excl += s[q] & S::VAL;
      if (flag == S::INC) {
        done = true;
        break;
      }
    }
    if (done) break;
    if (q == 0) lb_pause();
    j -= q;
  }
  st_agent(mine, (ST)(S::INC | (ST)(excl + count)));
  return excl;
}


// Split form of lookback() for overlapping the first status read with other
// work: lookback_begin publishes the aggregate and issues the read of the
// direct predecessor; lookback_end consumes it, walks further if needed and
// publishes the inclusive prefix.
template <int ND, typename ST>
__device__ __forceinline__ ST lookback_begin(ST* __restrict__ status, uint32_t tile, uint32_t first_tile, uint32_t t,
                                             uint64_t count) {
  using S = Status<ST>;
  ST* mine = status + (uint64_t)tile * ND + t;
  if (tile == first_tile) {
    st_agent(mine, (ST)(S::INC | (ST)count));
    return (ST)0;
  }
  st_agent(mine, (ST)(S::AGG | (ST)count));
  return ld_agent(status + (uint64_t)(tile - 1) * ND + t);
}

template <int ND, typename ST>
__device__ __forceinline__ uint64_t lookback_end(ST* __restrict__ status, uint32_t tile, uint32_t first_tile,
                                                 uint32_t t, uint64_t count, ST first_read) {
  using S = Status<ST>;
  if (tile == first_tile) return 0;
  ST* mine = status + (uint64_t)tile * ND + t;
  uint64_t excl = 0;
  int64_t j = (int64_t)tile - 1;
  ST s0 = first_read;
  for (;;) {
    if ((s0 & S::FLAGS) != 0) break;
    lb_pause();
    s0 = ld_agent(status + (uint64_t)j * ND + t);
  }
  excl += s0 & S::VAL;
  if ((s0 & S::FLAGS) == S::INC) {
    st_agent(mine, (ST)(S::INC | (ST)(excl + count)));
    return excl;
  }
  --j;
  for (;;) {
    ST s[LB_WIDTH];
#pragma unroll
    for (int q = 0; q < LB_WIDTH; ++q)
      s[q] = (j - q >= (int64_t)first_tile) ? ld_agent(status + (uint64_t)(j - q) * ND + t) : (ST)0;
    int q = 0;
    bool done = false;
    for (; q < LB_WIDTH && j - q >= (int64_t)first_tile; ++q) {
      const ST flag = s[q] & S::FLAGS;
      if (flag == 0) break;
      excl += s[q] & S::VAL;
      if (flag == S::INC) {
        done = true;
        break;
      }
    }
    if (done) break;
    if (q == 0) lb_pause();
    j -= q;
  }
  st_agent(mine, (ST)(S::INC | (ST)(excl + count)));
  return excl;
}

}  // namespace ahs
