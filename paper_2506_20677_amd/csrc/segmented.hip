// Batched segmented sort on gfx950: many independent arrays in one call.
// Segments of at most SS_CAP keys are handled wholly in LDS by one fused
// kernel (load, stable sort, features, decision, store); larger segments go
// through the sample-sort levels and get their features from runs of equal
// bins in their sorted output.  Features are permutation-invariant, so
// computing them after sorting gives the same values as before.
#include "blocksort.hpp"
#include "segmented.hpp"

namespace ahs {

// Decision engine of Sec. III-A on the device.  thr[B] = h_ratio * log2(B)
// is tabulated by the host with the host's log2, so the radix test compares
// exactly as the host decision engine does.
__device__ __forceinline__ uint8_t seg_fsm(uint64_t n, uint64_t span, uint32_t nbins, double H, const SegConfig& c,
                                           const double* __restrict__ thr) {
  if (n <= c.n_small) return 4;                  // INSERTION
  if (span <= c.k_count - 1) return 1;           // COUNTING
  if (span >= c.k_radix && H < thr[nbins]) return 2;  // RADIX
  return 3;                                      // QUICK
}

// Mapped-key bounds of the non-NaN values: map(-inf) .. map(+inf).
template <typename K> struct NanBounds;
template <> struct NanBounds<uint32_t> {
  static constexpr uint32_t lo = 0x007FFFFFu, hi = 0xFF800000u;
};
template <> struct NanBounds<uint64_t> {
  static constexpr uint64_t lo = 0x000FFFFFFFFFFFFFull, hi = 0xFFF0000000000000ull;
};

__device__ __forceinline__ void shift_nbins(uint64_t span, uint32_t& shift, uint32_t& nbins) {
  const int bl = bitlen64(span);
  shift = bl > 16 ? (uint32_t)(bl - 16) : 0u;
  nbins = (uint32_t)(span >> shift) + 1u;
}

// ------------------------------------------------------------------ classify
__global__ __launch_bounds__(256) void k_seg_classify(const uint64_t* __restrict__ offs, uint32_t nseg,
                                                      uint64_t n_total, uint32_t* __restrict__ small_ids,
                                                      SsSeg* __restrict__ large, SsSeg* __restrict__ large_copy,
                                                      uint32_t* __restrict__ large_ids,
                                                      SegCounters* __restrict__ ctr) {
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  if (s == 0 && offs[nseg] != n_total) atomicOr(&ctr->bad, 1u);
  if (s >= nseg) return;
  const uint64_t a = offs[s], b = offs[s + 1];
  if (b < a || b > n_total || b - a > 0xFFFFFFFFull) {
    atomicOr(&ctr->bad, 2u);
    return;
  }
  const uint64_t size = b - a;
  if (size <= (uint64_t)SS_CAP) {
    small_ids[atomicAdd(&ctr->nsmall, 1u)] = s;
  } else {
    const uint32_t i = atomicAdd(&ctr->nlarge, 1u);
    SsSeg g;
    g.start = a;
    g.size = (uint32_t)size;
    g.first_tile = 0;
    large[i] = g;
    large_copy[i] = g;
    large_ids[i] = s;
    atomicAdd(&ctr->large_keys, (unsigned long long)size);
    atomicMax(&ctr->max_large, (uint32_t)size);
  }
}

// ------------------------------------------------------------------ small segments, fused
template <int KK, bool PAY>
__global__ __launch_bounds__(SS_THREADS) void k_seg_small(SegArgs a) {
  using K = typename KeyTraits<KK>::K;
  __shared__ BlockSortSmem<K, PAY> sm;
  const uint32_t s = a.small_ids[blockIdx.x];
  const uint64_t base = a.offs[s];
  const uint32_t size = (uint32_t)(a.offs[s + 1] - base);
  const int t = threadIdx.x;
  const K* __restrict__ kin = (const K*)a.kin + base;
  K* __restrict__ kout = (K*)a.kout + base;
  lds_load_mapped<KK, PAY>(sm, kin, PAY ? a.vin + base : nullptr, size, true);
  K mn = 0, mx = 0;
  if (size > 0) lds_sort_loaded<K, PAY>(sm, size, mn, mx);
  for (uint32_t j = t; j < size; j += SS_THREADS) {
    K x = sm.keys[j];
    if constexpr (KeyTraits<KK>::FLT) x = funmap(x);
    kout[j] = x;
    if constexpr (PAY) a.vout[base + j] = sm.vals[j];
  }
  // features from the sorted keys (exclude NaNs, which sit at both ends)
  uint32_t nan = 0, lo = 0, hi = size;
  if constexpr (KeyTraits<KK>::FLT) {
    for (uint32_t j = t; j < size; j += SS_THREADS)
      nan += (sm.keys[j] < NanBounds<K>::lo || sm.keys[j] > NanBounds<K>::hi) ? 1u : 0u;
    nan = wave_sum(nan);
    if (lane_id() == 0) sm.scan[t / WAVE] = nan;
    __syncthreads();
    nan = 0;
    for (int i = 0; i < SS_THREADS / WAVE; ++i) nan += sm.scan[i];
    __syncthreads();
  }
  DevFeatures f = {};
  f.n = size;
  f.nan_count = nan;
  uint8_t chosen;
  if (nan) {
    chosen = SEG_STATUS_NAN;
  } else {
    if (size > 0) {
      mn = sm.keys[lo];
      mx = sm.keys[hi - 1];
    }
    f.min_key = mn;
    f.max_key = mx;
    f.span = (uint64_t)(mx - mn);
    shift_nbins(f.span, f.shift, f.nbins);
    f.exact = f.shift == 0;
    uint64_t carry = 0;
    double H = 0.0;
    if (size > 0)
      H = lds_run_entropy<K, PAY>(sm, size, 0, K(0), false, K(0), false, mn, f.shift, size, carry);
    f.entropy_bits = H < 0.0 ? 0.0 : H;
    f.entropy_ratio = f.nbins > 1 ? f.entropy_bits / log2((double)f.nbins) : 0.0;
    chosen = a.requested ? (uint8_t)a.requested : seg_fsm(size, f.span, f.nbins, f.entropy_bits, a.cfg, a.thr);
    if (size == 0) {
      f.nbins = 0;
      f.exact = 0;
    }
  }
  if (t == 0) {
    if (a.chosen) a.chosen[s] = chosen;
    if (a.feats) a.feats[s] = f;
  }
}

// ------------------------------------------------------------------ large segments: features after sorting
template <int KK>
__global__ __launch_bounds__(SS_THREADS) void k_seg_large(SegArgs a) {
  using K = typename KeyTraits<KK>::K;
  __shared__ BlockSortSmem<K, false> sm;
  const SsSeg g = a.large[blockIdx.x];
  const uint32_t s = a.large_ids[blockIdx.x];
  const K* __restrict__ keys = (const K*)a.kout + g.start;
  const uint32_t size = g.size;
  auto mapped = [&](uint64_t j) {
    K x = keys[j];
    if constexpr (KeyTraits<KK>::FLT) x = fmap(x);
    return x;
  };
  // NaNs occupy a prefix and a suffix of the sorted mapped order
  uint32_t lo = 0, hi = size;
  if constexpr (KeyTraits<KK>::FLT) {
    uint32_t l = 0, h = size;  // first index with mapped >= lo bound
    while (l < h) { const uint32_t m = (l + h) >> 1; if (mapped(m) < NanBounds<K>::lo) l = m + 1; else h = m; }
    lo = l;
    l = lo; h = size;  // first index with mapped > hi bound
    while (l < h) { const uint32_t m = (l + h) >> 1; if (mapped(m) > NanBounds<K>::hi) h = m; else l = m + 1; }
    hi = l;
  }
  DevFeatures f = {};
  f.n = size;
  f.nan_count = lo + (size - hi);
  uint8_t chosen;
  if (f.nan_count) {
    chosen = SEG_STATUS_NAN;
  } else {
    const K mn = mapped(0), mx = mapped(size - 1);
    f.min_key = mn;
    f.max_key = mx;
    f.span = (uint64_t)(mx - mn);
    shift_nbins(f.span, f.shift, f.nbins);
    f.exact = f.shift == 0;
    double H = 0.0;
    uint64_t carry = 0;
    for (uint32_t c0 = 0; c0 < size; c0 += SS_CAP) {
      const uint32_t cnt = size - c0 < (uint32_t)SS_CAP ? size - c0 : (uint32_t)SS_CAP;
      for (uint32_t j = threadIdx.x; j < cnt; j += SS_THREADS) sm.keys[j] = mapped(c0 + j);
      const K prev = c0 > 0 ? mapped(c0 - 1) : K(0);
      const K next = c0 + cnt < size ? mapped(c0 + cnt) : K(0);
      __syncthreads();
      H += lds_run_entropy<K, false>(sm, cnt, c0, prev, c0 > 0, next, c0 + cnt < size, mn, f.shift, size, carry);
    }
    f.entropy_bits = H < 0.0 ? 0.0 : H;
    f.entropy_ratio = f.nbins > 1 ? f.entropy_bits / log2((double)f.nbins) : 0.0;
    chosen = a.requested ? (uint8_t)a.requested : seg_fsm(size, f.span, f.nbins, f.entropy_bits, a.cfg, a.thr);
  }
  if (threadIdx.x == 0) {
    if (a.chosen) a.chosen[s] = chosen;
    if (a.feats) a.feats[s] = f;
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_seg_classify(const uint64_t* offs, uint32_t nseg, uint64_t n_total, uint32_t* small_ids, SsSeg* large,
                               SsSeg* large_copy, uint32_t* large_ids, SegCounters* ctr, hipStream_t s) {
  const uint32_t nb = (nseg + 256) / 256;
  k_seg_classify<<<nb, 256, 0, s>>>(offs, nseg, n_total, small_ids, large, large_copy, large_ids, ctr);
  return hipGetLastError();
}

hipError_t launch_seg_small(int kk, int with_vals, const SegArgs& a, uint32_t nsmall, hipStream_t s) {
  if (nsmall == 0) return hipSuccess;
  switch (kk * 2 + (with_vals ? 1 : 0)) {
    case KK_U32 * 2: k_seg_small<KK_U32, false><<<nsmall, SS_THREADS, 0, s>>>(a); break;
    case KK_U32 * 2 + 1: k_seg_small<KK_U32, true><<<nsmall, SS_THREADS, 0, s>>>(a); break;
    case KK_U64 * 2: k_seg_small<KK_U64, false><<<nsmall, SS_THREADS, 0, s>>>(a); break;
    case KK_U64 * 2 + 1: k_seg_small<KK_U64, true><<<nsmall, SS_THREADS, 0, s>>>(a); break;
    case KK_F32 * 2: k_seg_small<KK_F32, false><<<nsmall, SS_THREADS, 0, s>>>(a); break;
    case KK_F32 * 2 + 1: k_seg_small<KK_F32, true><<<nsmall, SS_THREADS, 0, s>>>(a); break;
    case KK_F64 * 2: k_seg_small<KK_F64, false><<<nsmall, SS_THREADS, 0, s>>>(a); break;
    case KK_F64 * 2 + 1: k_seg_small<KK_F64, true><<<nsmall, SS_THREADS, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_seg_large(int kk, const SegArgs& a, uint32_t nlarge, hipStream_t s) {
  if (nlarge == 0) return hipSuccess;
  switch (kk) {
    case KK_U32: k_seg_large<KK_U32><<<nlarge, SS_THREADS, 0, s>>>(a); break;
    case KK_U64: k_seg_large<KK_U64><<<nlarge, SS_THREADS, 0, s>>>(a); break;
    case KK_F32: k_seg_large<KK_F32><<<nlarge, SS_THREADS, 0, s>>>(a); break;
    case KK_F64: k_seg_large<KK_F64><<<nlarge, SS_THREADS, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ahs
