// In-LDS stable sort of up to CAP keys by one workgroup of NT threads, and
// the run statistics of a sorted key array (for features computed after
// sorting).  NT >= 256 (one thread per digit) and CAP / NT <= 16.
#pragma once

#include "onesweep.hpp"
#include "samplesort.hpp"

namespace ahs {

template <typename K, bool PAY, int CAP = SS_CAP, int NT = SS_THREADS>
struct BlockSortSmem {
  static_assert(NT >= 256 && CAP % NT == 0 && CAP / NT <= 16, "block sort shape");
  static constexpr int cap = CAP, nt = NT, nw = NT / WAVE;
  // rank state of each wave, then each pass's position table, the u16
  // destinations of the group ranks or the run starts of lds_run_entropy
  static constexpr size_t RANK_BYTES = sizeof(RankLds<256>) * (NT / WAVE);
  static constexpr size_t SCRATCH_BYTES = RANK_BYTES > sizeof(uint32_t) * CAP ? RANK_BYTES : sizeof(uint32_t) * CAP;
  __align__(16) unsigned char scratch[SCRATCH_BYTES];
  __device__ RankLds<256>* rank() { return reinterpret_cast<RankLds<256>*>(scratch); }
  __device__ uint32_t (*pos())[256] { return reinterpret_cast<uint32_t(*)[256]>(scratch); }
  K keys[CAP];
  uint32_t vals[PAY ? CAP : 1];
  uint32_t scan[NT / WAVE + 1];
  K red[2][NT / WAVE];
  double dred[NT / WAVE];
  uint32_t gmax[NT / WAVE];
  uint32_t grp[2][256];  // top-digit groups: start and count
  uint32_t misc[4];
};

// Loads `size` keys (mapping raw float bit patterns when `raw`) and
// payloads into LDS.  Every load of the thread is issued before the first
// LDS store (a load-store loop waits out one memory latency per key).
// Ends with a barrier.
template <int KK, bool PAY, typename SM>
__device__ __forceinline__ void lds_load_mapped(SM& sm, const typename KeyTraits<KK>::K* __restrict__ src,
                                                const uint32_t* __restrict__ vsrc, uint32_t size, bool raw) {
  using K = typename KeyTraits<KK>::K;
  constexpr int IPT = SM::cap / SM::nt;
  const uint32_t t = threadIdx.x;
  K x[IPT];
  uint32_t v[IPT];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint32_t j = t + (uint32_t)i * SM::nt;
    if (j < size) {
      x[i] = src[j];
      if constexpr (PAY) v[i] = vsrc[j];
    }
  }
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint32_t j = t + (uint32_t)i * SM::nt;
    if (j < size) {
      K y = x[i];
      if constexpr (key_mapped<KK>) y = raw ? map_key<KK>(y) : y;
      sm.keys[j] = y;
      if constexpr (PAY) sm.vals[j] = v[i];
    }
  }
  __syncthreads();
}

// Stable rank sort of sm.keys[0, size), size <= NT: thread t holds key t
// and counts the keys that sort before it, smaller keys and equal keys at
// lower indices (keys of lower waves: <=; of higher waves: <; of its own
// wave: by lane).  One pass of size^2 / NT broadcast reads and compares: for
// small buckets this beats the LSD passes, whose state clearing, scans and
// barriers cost about the same at any size.  Ends with a barrier.
template <typename K, bool PAY, int CAP, int NT>
__device__ __forceinline__ void lds_rank_sort(BlockSortSmem<K, PAY, CAP, NT>& sm, uint32_t size) {
  const uint32_t t = threadIdx.x;
  const uint32_t wlo = t / WAVE * WAVE;
  K my = ~K(0);
  uint32_t mv = 0, rank = 0;
  if (wlo < size) {  // uniform over the wave
    if (t < size) {
      my = sm.keys[t];
      if constexpr (PAY) mv = sm.vals[t];
    }
    const uint32_t whi = wlo + WAVE < size ? wlo + WAVE : size;
#pragma unroll 8
    for (uint32_t j = 0; j < wlo; ++j) rank += sm.keys[j] <= my ? 1u : 0u;
    for (uint32_t j = wlo; j < whi; ++j) {
      const K x = sm.keys[j];
      rank += (x < my || (x == my && j < t)) ? 1u : 0u;
    }
#pragma unroll 8
    for (uint32_t j = whi; j < size; ++j) rank += sm.keys[j] < my ? 1u : 0u;
  }
  __syncthreads();
  if (t < size) {
    sm.keys[rank] = my;
    if constexpr (PAY) sm.vals[rank] = mv;
  }
  __syncthreads();
}

// Largest bucket the block sort ranks in one pass (one key per thread).
constexpr uint32_t LDS_RANK_SORT_MAX = 512;
// Largest group of equal top digits ranked by comparisons after a top-digit
// pass (spans over 16 bits).
#ifndef AHS_GROUP_RANK_MAX
#define AHS_GROUP_RANK_MAX 64
#endif
constexpr uint32_t LDS_GROUP_RANK_MAX = AHS_GROUP_RANK_MAX;
#ifndef AHS_GROUP_RANK_MIN_BITS
#define AHS_GROUP_RANK_MIN_BITS 24
#endif
constexpr int LDS_GROUP_RANK_MIN_BITS = AHS_GROUP_RANK_MIN_BITS;  // spans of more bits try the group ranks

// Stable sort of sm.keys[0, size) (mapped keys) by 8-bit digits of
// (key - min): a rank sort when the keys fit one per thread; over 16 bits of
// span a top-digit pass and ranks inside its groups when they are small;
// otherwise as many LSD passes as the span needs.  Payloads move along.
// Returns min and max (mapped).  Ends with a barrier.
template <typename K, bool PAY, int CAP, int NT>
__device__ __forceinline__ void lds_sort_loaded(BlockSortSmem<K, PAY, CAP, NT>& sm, uint32_t size, K& out_min,
                                                K& out_max) {
  constexpr int IPT = CAP / NT;
  constexpr int NW = NT / WAVE;
  const int t = threadIdx.x, w = t / WAVE, lane = lane_id();
  K mn = ~K(0), mx = K(0);
  for (uint32_t j = t; j < size; j += NT) {
    const K x = sm.keys[j];
    mn = x < mn ? x : mn;
    mx = x > mx ? x : mx;
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  if (lane == 0) { sm.red[0][w] = mn; sm.red[1][w] = mx; }
  __syncthreads();
  mn = sm.red[0][0];
  mx = sm.red[1][0];
#pragma unroll
  for (int i = 1; i < NW; ++i) {
    mn = sm.red[0][i] < mn ? sm.red[0][i] : mn;
    mx = sm.red[1][i] > mx ? sm.red[1][i] : mx;
  }
  out_min = mn;
  out_max = mx;
  const int npass = (bitlen64((uint64_t)(mx - mn)) + 7) / 8;
  if (npass > 0 && size <= (uint32_t)NT && size <= LDS_RANK_SORT_MAX) {
    lds_rank_sort(sm, size);
    return;
  }

  // the keys are spread over all waves: wave w ranks the `per` items
  // [w * per * WAVE, (w + 1) * per * WAVE) in (item, lane) order, so ranks
  // stay stable, and a bucket half the capacity gives every wave half its
  // items (the serial rank steps of a wave are per item).  Items past
  // `size` hold only padding, which sorts last and is never read back.
  const uint32_t per = (size + NT - 1) / NT;
  const uint32_t wbase = (uint32_t)w * WAVE * per;
  const uint32_t wend = wbase + WAVE * per < size ? wbase + WAVE * per : size;
  const int nv = wend > wbase ? (int)((wend - wbase + WAVE - 1) / WAVE) : 0;

  // One stable pass by the 8-bit digit ((key - min) >> shift) & 255.  With
  // gmax > 0 the pass is abandoned before it moves a key when some digit
  // holds more than gmax keys (returns false); it then records every digit's
  // group (start, count) in sm.grp.
  auto pass = [&](uint32_t shift, uint32_t gmax) -> bool {
    K k[IPT];
    uint32_t v[IPT];
    uint32_t d[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t idx = wbase + (uint32_t)i * WAVE + lane;
      if (i < nv && idx < size) {
        k[i] = sm.keys[idx];
        if constexpr (PAY) v[i] = sm.vals[idx];
        d[i] = (uint32_t)(((k[i] - mn) >> shift) & 255u);
      } else {
        k[i] = ~K(0);
        if constexpr (PAY) v[i] = 0;
        d[i] = 255u;
      }
    }
    // the previous pass's position table overlays the rank state: clear it whole
    rank_clear<256, NT>(sm.rank(), NW);
    __syncthreads();
    uint32_t r[IPT];
    rank_wave_items<IPT>(d, r, sm.rank()[w], nv);
    __syncthreads();
    // per-wave exclusive prefixes of digit t in registers; after the scan's
    // first barrier (every count read) a dense per-(wave, digit) table of
    // tile positions overlays the rank state: one LDS read per key
    uint32_t cnt = 0, wpre[NW];
    if (t < 256) {
#pragma unroll
      for (int u = 0; u < NW; ++u) {
        wpre[u] = cnt;
        cnt += sm.rank()[u].count[t];
      }
    }
    if (gmax) {
      const uint32_t m = wave_max(t < 256 ? cnt : 0u);
      if (lane == 0) sm.gmax[w] = m;
      __syncthreads();
      uint32_t big = 0;
#pragma unroll
      for (int u = 0; u < NW; ++u) big = sm.gmax[u] > big ? sm.gmax[u] : big;
      if (big > gmax) return false;  // every count has been read: the next pass may clear them
    }
    uint32_t total;
    const uint32_t tstart = block_excl_scan<NT>(t < 256 ? cnt : 0u, sm.scan, total);
    uint32_t(*pos)[256] = sm.pos();
    static_assert(sizeof(uint32_t) * NW * 256 <= BlockSortSmem<K, PAY, CAP, NT>::SCRATCH_BYTES, "position table fits");
    if (t < 256) {
#pragma unroll
      for (int u = 0; u < NW; ++u) pos[u][t] = wpre[u] + tstart;
      if (gmax) {
        sm.grp[0][t] = tstart;
        sm.grp[1][t] = cnt;
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      if (i < nv) {
        const uint32_t lp = pos[w][d[i]] + r[i];
        if (lp < (uint32_t)CAP) {
          sm.keys[lp] = k[i];
          if constexpr (PAY) sm.vals[lp] = v[i];
        }
      }
    }
    __syncthreads();
    return true;
  };

  const int bits = bitlen64((uint64_t)(mx - mn));
  if (bits > LDS_GROUP_RANK_MIN_BITS) {
    // Wide spans: one pass by the top 8 bits, then, if no group of
    // equal top digits holds more than LDS_GROUP_RANK_MAX keys, each key is
    // ranked inside its group (the keys before it that are smaller, or equal
    // at a lower index: stable), instead of ceil(bits / 8) LSD passes.
    const uint32_t shift = (uint32_t)bits - 8u;
    if (pass(shift, LDS_GROUP_RANK_MAX)) {
      // destinations first (u16, in the free scratch), then the moves: a
      // thread holds no per-item rank state, only its keys while they move
      uint16_t* s_dst = reinterpret_cast<uint16_t*>(sm.scratch);
      static_assert(sizeof(uint16_t) * CAP <= sizeof(sm.scratch), "destinations fit in the scratch");
      for (uint32_t j = (uint32_t)t; j < size; j += NT) {
        const K x = sm.keys[j];
        const uint32_t dg = (uint32_t)(((x - mn) >> shift) & 255u);
        const uint32_t gs = sm.grp[0][dg];
        const uint32_t ge = gs + sm.grp[1][dg] < size ? gs + sm.grp[1][dg] : size;
        uint32_t rk = 0;
        uint32_t q = gs;
        for (; q + 4u <= ge; q += 4u) {  // four reads in flight
          const K y0 = sm.keys[q], y1 = sm.keys[q + 1], y2 = sm.keys[q + 2], y3 = sm.keys[q + 3];
          rk += (y0 < x || (y0 == x && q < j)) ? 1u : 0u;
          rk += (y1 < x || (y1 == x && q + 1u < j)) ? 1u : 0u;
          rk += (y2 < x || (y2 == x && q + 2u < j)) ? 1u : 0u;
          rk += (y3 < x || (y3 == x && q + 3u < j)) ? 1u : 0u;
        }
        for (; q < ge; ++q) {
          const K y = sm.keys[q];
          rk += (y < x || (y == x && q < j)) ? 1u : 0u;
        }
        s_dst[j] = (uint16_t)(gs + rk);
      }
      __syncthreads();
      K k[IPT];
      uint32_t v[IPT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const uint32_t j = (uint32_t)t + (uint32_t)i * NT;
        if (j < size) {
          k[i] = sm.keys[j];
          if constexpr (PAY) v[i] = sm.vals[j];
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const uint32_t j = (uint32_t)t + (uint32_t)i * NT;
        if (j < size) {
          const uint32_t o = s_dst[j];
          sm.keys[o] = k[i];
          if constexpr (PAY) sm.vals[o] = v[i];
        }
      }
      __syncthreads();
      return;
    }
  }
  for (int p = 0; p < npass; ++p) pass(8u * (uint32_t)p, 0u);
}

// Sum over the runs of equal bins (key - kmin) >> shift inside one chunk of
// a sorted array of mapped keys: each run of c keys of a segment of n keys
// contributes -(c/n) log2(c/n).  The chunk holds cnt keys (in LDS) starting
// at segment position pos0; prev_key / next_key are the keys just before
// and after the chunk (has_prev / has_next false at the segment ends).
// carry_start is the segment position where the run open at the chunk's
// start began; it is updated to the start of the run open at the chunk's end.
// Returns the block's FP64 sum (valid in every thread).  Uses sm.scratch as
// scratch for run starts (CAP u32 entries fit in it).
template <typename K, bool PAY, int CAP, int NT>
__device__ __forceinline__ double lds_run_entropy(BlockSortSmem<K, PAY, CAP, NT>& sm, uint32_t cnt, uint64_t pos0,
                                                  K prev_key, bool has_prev, K next_key, bool has_next, K kmin,
                                                  uint32_t shift, uint64_t n, uint64_t& carry_start) {
  constexpr int CH = CAP / NT;  // consecutive positions per thread
  const int t = threadIdx.x;
  uint32_t* s_start = reinterpret_cast<uint32_t*>(sm.scratch);  // run starts (chunk-relative)
  const uint32_t j0 = (uint32_t)t * CH;
  auto binof = [&](K x) { return (uint64_t)((x - kmin) >> shift); };
  // run starts in my positions
  uint32_t nst = 0;
  uint32_t startbits = 0;
  for (int q = 0; q < CH; ++q) {
    const uint32_t j = j0 + q;
    if (j >= cnt) break;
    bool st;
    if (j == 0) st = !has_prev || binof(prev_key) != binof(sm.keys[0]);
    else st = binof(sm.keys[j - 1]) != binof(sm.keys[j]);
    if (st) { ++nst; startbits |= 1u << q; }
  }
  uint32_t total;
  uint32_t r = block_excl_scan<NT>(nst, sm.scan, total);
  for (int q = 0; q < CH; ++q)
    if (startbits >> q & 1u) s_start[r++] = j0 + q;
  __syncthreads();
  const uint64_t carry_in = carry_start;
  double acc = 0.0;
  const double inv_n = 1.0 / (double)n;
  r = r - nst;  // runs started before my first position
  for (int q = 0; q < CH; ++q) {
    const uint32_t j = j0 + q;
    if (j >= cnt) break;
    if (startbits >> q & 1u) ++r;
    bool end;
    if (j + 1 == cnt) end = !has_next || binof(next_key) != binof(sm.keys[j]);
    else end = binof(sm.keys[j + 1]) != binof(sm.keys[j]);
    if (end) {
      const uint64_t start = r == 0 ? carry_in : pos0 + s_start[r - 1];
      const double c = (double)(pos0 + j + 1 - start);
      const double p = c * inv_n;
      acc -= p * log2(p);
    }
  }
  // new carry: start of the last run in the chunk
  if (total > 0) carry_start = pos0 + s_start[total - 1];
  acc = wave_sum(acc);
  if (lane_id() == 0) sm.dred[t / WAVE] = acc;
  __syncthreads();
  double sum = 0.0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) sum += sm.dred[i];
  __syncthreads();
  return sum;
}

}  // namespace ahs
