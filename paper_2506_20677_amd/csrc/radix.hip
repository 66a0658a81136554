// LSD radix sort pass on gfx950 (Sec. III-G, base 256; eq. (4) digit
// count): one stable single-pass scatter of all keys by the 8-bit digit
// ((key - min) >> shift) & 255.  Global digit offsets come from the upfront
// digit histogram; per-tile offsets from a decoupled look-back across tiles;
// keys are staged in LDS in digit order so the global writes are runs of
// consecutive addresses.
#include "onesweep.hpp"

namespace ahs {

template <int KK, bool PAY, int IPT>
__global__ __launch_bounds__(OS_THREADS) void k_onesweep(OnesweepArgs a) {
  using K = typename KeyTraits<KK>::K;
  constexpr int TILE = OS_THREADS * IPT;
  constexpr int NW = OS_WAVES;
  __shared__ uint64_t s_mask[NW][256];
  __shared__ uint32_t s_whist[NW][256];
  __shared__ uint32_t s_tstart[256];
  __shared__ uint32_t s_dbase[256];
  __shared__ K s_keys[TILE];
  __shared__ uint32_t s_vals[PAY ? TILE : 1];
  __shared__ uint8_t s_dig[TILE];
  __shared__ uint32_t s_scan[NW + 1];
  __shared__ uint32_t s_tile;

  const int t = threadIdx.x, w = t / WAVE, lane = lane_id();
  for (int i = t; i < NW * 256; i += OS_THREADS) {
    (&s_mask[0][0])[i] = 0ull;
    (&s_whist[0][0])[i] = 0u;
  }
  if (t == 0) s_tile = add_agent(a.tile_counter, 1u);
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint64_t tbase = (uint64_t)tile * TILE;
  const uint64_t wbase = tbase + (uint64_t)w * WAVE * IPT;
  const K* __restrict__ src = (const K*)a.src;
  const K kmin = (K)a.kmin;

  K k[IPT];
  uint32_t v[IPT];
  uint32_t d[IPT];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint64_t idx = wbase + (uint64_t)i * WAVE + lane;
    if (idx < a.n) {
      K x = src[idx];
      if constexpr (KeyTraits<KK>::FLT) x = a.map_in ? fmap(x) : x;
      k[i] = x;
      if constexpr (PAY) v[i] = a.vsrc[idx];
      d[i] = (uint32_t)(((x - kmin) >> a.digit_shift) & 255u);
    } else {
      k[i] = ~K(0);
      if constexpr (PAY) v[i] = 0;
      d[i] = 255u;
    }
  }

  uint32_t r[IPT];
  rank_wave_items<IPT>(d, r, s_mask[w], s_whist[w]);
  __syncthreads();

  uint32_t cnt = wave_prefix_per_digit<NW>(s_whist);
  const uint64_t valid64 = a.n - tbase < (uint64_t)TILE ? a.n - tbase : (uint64_t)TILE;
  const uint32_t valid = (uint32_t)valid64;
  if (t == 255) cnt -= (uint32_t)TILE - valid;  // padding sorted last under digit 255
  uint32_t total;
  const uint32_t tstart = block_excl_scan<OS_THREADS>(t < 256 ? cnt : 0u, s_scan, total);
  if (t < 256) {
    s_tstart[t] = tstart;
    const uint64_t excl = lookback(a.status, tile, 0u, (uint32_t)t, cnt, a.epoch);
    s_dbase[t] = a.digit_offsets[t] + (uint32_t)excl;
  }
  __syncthreads();

#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint32_t lp = s_tstart[d[i]] + s_whist[w][d[i]] + r[i];
    if (lp < (uint32_t)TILE) {
      s_keys[lp] = k[i];
      if constexpr (PAY) s_vals[lp] = v[i];
      s_dig[lp] = (uint8_t)d[i];
    }
  }
  __syncthreads();

  K* __restrict__ dst = (K*)a.dst;
  for (uint32_t j = t; j < valid; j += OS_THREADS) {
    const uint32_t dj = s_dig[j];
    const uint32_t o = s_dbase[dj] + (j - s_tstart[dj]);
    if (o >= a.n) continue;  // unreachable with consistent digit counts
    K x = s_keys[j];
    if constexpr (KeyTraits<KK>::FLT) x = a.unmap_out ? funmap(x) : x;
    dst[o] = x;
    if constexpr (PAY) a.vdst[o] = s_vals[j];
  }
}

template <int KK, bool PAY>
static hipError_t onesweep_kk(const OnesweepArgs& a, hipStream_t s) {
  constexpr int IPT = sizeof(typename KeyTraits<KK>::K) == 4 ? 16 : 8;
  constexpr int TILE = OS_THREADS * IPT;
  const uint64_t tiles = (a.n + TILE - 1) / TILE;
  k_onesweep<KK, PAY, IPT><<<(unsigned)tiles, OS_THREADS, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_onesweep(int kk, int with_vals, const OnesweepArgs& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  switch (kk * 2 + (with_vals ? 1 : 0)) {
    case KK_U32 * 2: return onesweep_kk<KK_U32, false>(a, s);
    case KK_U32 * 2 + 1: return onesweep_kk<KK_U32, true>(a, s);
    case KK_U64 * 2: return onesweep_kk<KK_U64, false>(a, s);
    case KK_U64 * 2 + 1: return onesweep_kk<KK_U64, true>(a, s);
    case KK_F32 * 2: return onesweep_kk<KK_F32, false>(a, s);
    case KK_F32 * 2 + 1: return onesweep_kk<KK_F32, true>(a, s);
    case KK_F64 * 2: return onesweep_kk<KK_F64, false>(a, s);
    case KK_F64 * 2 + 1: return onesweep_kk<KK_F64, true>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ahs
