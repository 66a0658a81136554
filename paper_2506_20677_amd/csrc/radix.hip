// LSD radix sort pass on gfx950 (Sec. III-G, base 256; eq. (4) digit
// count): one stable single-pass scatter of all keys by the 8-bit digit
// ((key - min) >> shift) & 255.  Global digit offsets come from the upfront
// digit histogram; per-tile offsets from a decoupled look-back across tiles;
// keys are staged in LDS in digit order so the global writes are runs of
// consecutive addresses.
#include "onesweep.hpp"

namespace ahs {

template <int KK, bool PAY, int IPT, typename ST>
__global__ __launch_bounds__(OS_THREADS) void k_onesweep(OnesweepArgs a) {
  using K = typename KeyTraits<KK>::K;
  constexpr int TILE = OS_THREADS * IPT;
  constexpr int NW = OS_WAVES;
  // One LDS region holds in turn the rank state, the dense per-(wave,
  // digit) position table (written once every count has been read, after
  // the scan's first barrier) and the staged keys (once every key's tile
  // position is in a register).
  constexpr size_t SLOT_BYTES = sizeof(RankLds<256>) * NW;
  constexpr size_t KEY_BYTES = sizeof(K) * TILE;
  static_assert(sizeof(uint32_t) * NW * 256 <= SLOT_BYTES, "position table fits over the slots");
  __shared__ __align__(16) unsigned char s_raw[SLOT_BYTES > KEY_BYTES ? SLOT_BYTES : KEY_BYTES];
  RankLds<256>* s_rank = reinterpret_cast<RankLds<256>*>(s_raw);
  uint32_t(*s_pos)[256] = reinterpret_cast<uint32_t(*)[256]>(s_raw);
  K* s_keys = reinterpret_cast<K*>(s_raw);
  __shared__ uint32_t s_tstart[256];
  __shared__ uint32_t s_dadj[256];  // global position of the tile's key j with digit d: s_dadj[d] + j
  __shared__ uint32_t s_vals[PAY ? TILE : 1];
  __shared__ uint32_t s_scan[NW + 1];
  __shared__ uint32_t s_tile;

  const int t = threadIdx.x, w = t / WAVE, lane = lane_id();
  rank_clear<256, OS_THREADS>(s_rank, NW);
  if (t == 0) s_tile = add_agent(a.tile_counter, 1u);
  const uint32_t doff = t < 256 ? a.digit_offsets[t] : 0u;  // in flight early
  __syncthreads();
  const uint32_t tile = s_tile;
  const uint64_t tbase = (uint64_t)tile * TILE;
  const uint64_t wbase = tbase + (uint64_t)w * WAVE * IPT;
  const K* __restrict__ src = (const K*)a.src;
  const K kmin = (K)a.kmin;
  const uint32_t shift = a.digit_shift;
  const uint64_t last = a.n - 1;
  auto digit = [&](K x) { return (uint32_t)(((x - kmin) >> shift) & 255u); };

  // all loads in flight first (indices clamped); padding keys become the
  // largest key, which sorts last under digit 255 and is never written
  K k[IPT];
  uint32_t v[IPT];
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    const uint64_t idx = wbase + (uint64_t)i * WAVE + lane;
    k[i] = src[idx < a.n ? idx : last];
    if constexpr (PAY) v[i] = a.vsrc[idx < a.n ? idx : last];
  }
  const bool full = tbase + TILE <= a.n;
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    if constexpr (key_mapped<KK>) k[i] = a.map_in ? map_key<KK>(k[i]) : k[i];
    if (!full && wbase + (uint64_t)i * WAVE + lane >= a.n) k[i] = kmin + (K)(255ull << shift);
  }

  uint32_t r[IPT];
  {
    uint32_t d[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) d[i] = digit(k[i]);
    rank_wave_items<IPT>(d, r, s_rank[w]);
  }
  __syncthreads();

  // per-wave exclusive prefixes of digit t, kept in registers until the
  // tile's digit starts are known
  uint32_t cnt = 0, wpre[NW];
  if (t < 256) {
#pragma unroll
    for (int u = 0; u < NW; ++u) {
      wpre[u] = cnt;
      cnt += s_rank[u].count[t];
    }
  }
  const uint64_t valid64 = a.n - tbase < (uint64_t)TILE ? a.n - tbase : (uint64_t)TILE;
  const uint32_t valid = (uint32_t)valid64;
  if (t == 255) cnt -= (uint32_t)TILE - valid;
  uint32_t total;
  const uint32_t tstart = block_excl_scan<OS_THREADS>(t < 256 ? cnt : 0u, s_scan, total);
  ST pred = 0;
  if (t < 256) {
    s_tstart[t] = tstart;
    pred = lookback_begin<256, ST>((ST*)a.status, tile, 0u, (uint32_t)t, cnt);
    // dense table of tile positions per (wave, digit): one LDS read per key
    // below instead of two strided ones
#pragma unroll
    for (int u = 0; u < NW; ++u) s_pos[u][t] = wpre[u] + tstart;
  }
  __syncthreads();
  // stage keys in digit order while the predecessor's status is in flight
#pragma unroll
  for (int i = 0; i < IPT; ++i) r[i] += s_pos[w][digit(k[i])];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IPT; ++i) {
    if (r[i] < (uint32_t)TILE) {
      s_keys[r[i]] = k[i];
      if constexpr (PAY) s_vals[r[i]] = v[i];
    }
  }
  if (t < 256) {
    const uint64_t excl = lookback_end<256, ST>((ST*)a.status, tile, 0u, (uint32_t)t, cnt, pred);
    s_dadj[t] = doff + (uint32_t)excl - tstart;  // modulo 2^32; + j lands in [0, n)
  }
  __syncthreads();

  K* __restrict__ dst = (K*)a.dst;
  auto put = [&](uint32_t j, K x, uint32_t o) {
    if (o >= a.n) return;  // unreachable with consistent digit counts
    if constexpr (key_mapped<KK>) x = a.unmap_out ? unmap_key<KK>(x) : x;
    dst[o] = x;
    if constexpr (PAY) a.vdst[o] = s_vals[j];
  };
  if (valid == (uint32_t)TILE) {
    // full tile: all LDS reads first, then the stores
    K x[IPT];
    uint32_t o[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) x[i] = s_keys[t + i * OS_THREADS];
#pragma unroll
    for (int i = 0; i < IPT; ++i) o[i] = s_dadj[digit(x[i])] + (uint32_t)(t + i * OS_THREADS);
#pragma unroll
    for (int i = 0; i < IPT; ++i) put((uint32_t)(t + i * OS_THREADS), x[i], o[i]);
  } else {
    for (uint32_t j = t; j < valid; j += OS_THREADS) {
      const K x = s_keys[j];
      put(j, x, s_dadj[digit(x)] + j);
    }
  }
}

template <int KK, bool PAY>
static hipError_t onesweep_kk(const OnesweepArgs& a, hipStream_t s) {
  constexpr int IPT = sizeof(typename KeyTraits<KK>::K) == 4 ? (PAY ? OS_IPT32P : OS_IPT32)
                                                            : (PAY ? OS_IPT64P : OS_IPT64);
  constexpr int TILE = OS_THREADS * IPT;
  const uint64_t tiles = (a.n + TILE - 1) / TILE;
  if (a.n < STATUS32_MAX_N)
    k_onesweep<KK, PAY, IPT, uint32_t><<<(unsigned)tiles, OS_THREADS, 0, s>>>(a);
  else
    k_onesweep<KK, PAY, IPT, uint64_t><<<(unsigned)tiles, OS_THREADS, 0, s>>>(a);
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
    case KK_I32 * 2: return onesweep_kk<KK_I32, false>(a, s);
    case KK_F32 * 2 + 1: return onesweep_kk<KK_F32, true>(a, s);
    case KK_I32 * 2 + 1: return onesweep_kk<KK_I32, true>(a, s);
    case KK_F64 * 2: return onesweep_kk<KK_F64, false>(a, s);
    case KK_I64 * 2: return onesweep_kk<KK_I64, false>(a, s);
    case KK_F64 * 2 + 1: return onesweep_kk<KK_F64, true>(a, s);
    case KK_I64 * 2 + 1: return onesweep_kk<KK_I64, true>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ahs
