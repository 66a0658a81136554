// Batched segmented sort on gfx950: many independent arrays in one call.
// Segments of at most SS_CAP keys are queued by size class and handled
// wholly in LDS by one fused kernel per class (load, stable sort, features,
// decision, store); larger segments go through the sample-sort levels and
// get their features from runs of equal bins in their sorted output.
// Features are permutation-invariant, so computing them after sorting gives
// the same values as before.  Every kernel reads its work count from the
// device, so the whole batch can be enqueued without a host round trip.
#include "blocksort.hpp"
#include "segmented.hpp"

namespace ahs {

// Mapped-key bounds of the non-NaN values: map(-inf) .. map(+inf).
template <typename K> struct NanBounds;
template <> struct NanBounds<uint32_t> {
  static constexpr uint32_t lo = 0x007FFFFFu, hi = 0xFF800000u;
};
template <> struct NanBounds<uint64_t> {
  static constexpr uint64_t lo = 0x000FFFFFFFFFFFFFull, hi = 0xFFF0000000000000ull;
};

// ------------------------------------------------------------------ classify
__global__ __launch_bounds__(256) void k_seg_classify(const uint64_t* __restrict__ offs, uint32_t nseg,
                                                      uint64_t n_total, uint32_t* __restrict__ queues, uint32_t qcap,
                                                      SegLarge* __restrict__ linfo, SsSeg* __restrict__ large,
                                                      uint32_t* __restrict__ large_ids,
                                                      SegCounters* __restrict__ ctr) {
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  if (s == 0 && offs[nseg] != n_total) atomicOr(&ctr->bad, SEG_ERR_OFFSETS);
  if (s >= nseg) return;
  const uint64_t a = offs[s], b = offs[s + 1];
  if (b < a || b > n_total || b - a > 0xFFFFFFFFull) {
    atomicOr(&ctr->bad, SEG_ERR_OFFSETS);
    return;
  }
  const uint64_t size = b - a;
  if (size <= (uint64_t)SS_CAP) {
    int c = 0;
    while (size > SEG_CLASS_CAP[c]) ++c;
    queues[(size_t)c * qcap + atomicAdd(&ctr->nclass[c], 1u)] = s;
    atomicAdd(&ctr->small_keys, (unsigned long long)size);
  } else {
    const uint32_t i = atomicAdd(&ctr->nlarge, 1u);
    SsSeg g;
    g.start = a;
    g.size = (uint32_t)size;
    g.first_tile = 0;
    large[i] = g;
    SegLarge L;
    L.mn = ~0ull;
    L.mx = 0ull;
    L.nan = 0u;
    L.pad = 0u;
    linfo[i] = L;
    large_ids[i] = s;
    atomicAdd(&ctr->large_keys, (unsigned long long)size);
    atomicMax(&ctr->max_large, (uint32_t)size);
  }
}

__global__ void k_seg_gate(const SegCounters* __restrict__ ctr, SsCounters* __restrict__ rec_chunks) {
  if (threadIdx.x == 0) {
    const uint32_t nl = ctr->bad ? 0u : ctr->nlarge;
    rec_chunks->nsegs_next = nl;
  }
}

// ------------------------------------------------------------------ small segments, fused
template <int KK, bool PAY, int CAP, int NT>
__global__ __launch_bounds__(NT) void k_seg_small(SegArgs a, int cls) {
  using K = typename KeyTraits<KK>::K;
  __shared__ BlockSortSmem<K, PAY, CAP, NT> sm;
  const uint32_t count = a.ctr->bad ? 0u : a.ctr->nclass[cls];
  const uint32_t* __restrict__ queue = a.queues + (size_t)cls * a.qcap;
  const int t = threadIdx.x;
  for (uint32_t q = blockIdx.x; q < count; q += gridDim.x) {
    __syncthreads();  // the previous segment's LDS contents are consumed
    const uint32_t s = queue[q];
    const uint64_t base = a.offs[s];
    const uint32_t size = (uint32_t)(a.offs[s + 1] - base);
    const K* __restrict__ kin = (const K*)a.kin + base;
    K* __restrict__ kout = (K*)a.kout + base;
    lds_load_mapped<KK, PAY>(sm, kin, PAY ? a.vin + base : nullptr, size, true);
    K mn = 0, mx = 0;
    if (size > 0) lds_sort_loaded(sm, size, mn, mx);
    for (uint32_t j = t; j < size; j += NT) {
      K x = sm.keys[j];
      if constexpr (key_mapped<KK>) x = unmap_key<KK>(x);
      kout[j] = x;
      if constexpr (PAY) a.vout[base + j] = sm.vals[j];
    }
    // features from the sorted keys (NaNs sit at both ends of the mapped order)
    uint32_t nan = 0;
    if constexpr (KeyTraits<KK>::FLT) {
      for (uint32_t j = t; j < size; j += NT)
        nan += (sm.keys[j] < NanBounds<K>::lo || sm.keys[j] > NanBounds<K>::hi) ? 1u : 0u;
      nan = wave_sum(nan);
      if (lane_id() == 0) sm.scan[t / WAVE] = nan;
      __syncthreads();
      nan = 0;
      for (int i = 0; i < NT / WAVE; ++i) nan += sm.scan[i];
      __syncthreads();
    }
    DevFeatures f = {};
    f.n = size;
    f.nan_count = nan;
    uint8_t chosen;
    if (nan) {
      chosen = SEG_STATUS_NAN;
    } else {
      f.min_key = mn;
      f.max_key = mx;
      f.span = (uint64_t)(mx - mn);
      shift_nbins(f.span, f.shift, f.nbins);
      f.exact = f.shift == 0;
      uint64_t carry = 0;
      double H = 0.0;
      if (size > 0) H = lds_run_entropy(sm, size, 0, K(0), false, K(0), false, mn, f.shift, size, carry);
      f.entropy_bits = H < 0.0 ? 0.0 : H;
      f.entropy_ratio = f.nbins > 1 ? f.entropy_bits / log2((double)f.nbins) : 0.0;
      chosen = a.requested ? (uint8_t)a.requested : seg_fsm(size, f.span, f.nbins, f.entropy_bits, a.cfg);
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
}

// ------------------------------------------------------------------ large segments: features after sorting
// NaN bounds of each sorted large segment: NaNs occupy a prefix and a suffix
// of the mapped order.  One thread per segment.
template <int KK>
__global__ __launch_bounds__(64) void k_seg_bounds(SegArgs a) {
  using K = typename KeyTraits<KK>::K;
  const uint32_t count = a.ctr->bad ? 0u : a.ctr->nlarge;
  for (uint32_t i = blockIdx.x * 64 + threadIdx.x; i < count; i += gridDim.x * 64) {
    const SsSeg g = a.large[i];
    uint32_t lo = 0, hi = g.size;
    if constexpr (KeyTraits<KK>::FLT) {
      const K* __restrict__ keys = (const K*)a.kout + g.start;
      uint32_t l = 0, h = g.size;  // first index with mapped >= map(-inf)
      while (l < h) {
        const uint32_t m = (l + h) >> 1;
        if (fmap(keys[m]) < NanBounds<K>::lo) l = m + 1; else h = m;
      }
      lo = l;
      h = g.size;  // first index with mapped > map(+inf)
      while (l < h) {
        const uint32_t m = (l + h) >> 1;
        if (fmap(keys[m]) > NanBounds<K>::hi) h = m; else l = m + 1;
      }
      hi = l;
    }
    a.bounds[2 * i] = lo;
    a.bounds[2 * i + 1] = hi;
  }
}

// Exclusive max over the threads of a workgroup (-1 identity).
template <int NT>
__device__ __forceinline__ int block_excl_max(int v, int* smem) {
  constexpr int NW = NT / WAVE;
  const int w = threadIdx.x / WAVE, l = lane_id();
  int inc = v;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const int o = __shfl_up(inc, d, WAVE);
    if (l >= d) inc = o > inc ? o : inc;
  }
  int ex = __shfl_up(inc, 1, WAVE);
  if (l == 0) ex = -1;
  if (l == WAVE - 1) smem[w] = inc;
  __syncthreads();
  int before = -1;
  for (int i = 0; i < w; ++i) before = smem[i] > before ? smem[i] : before;
  __syncthreads();
  return ex > before ? ex : before;
}

// Per chunk of a sorted large segment without NaNs: the entropy terms
// -(c/n) log2(c/n) of the runs of equal bins that END in the chunk.  A run
// that began before the chunk gets its start from a 64-way galloping search
// by one wave (bins ascend along the sorted segment).
template <int KK>
__global__ __launch_bounds__(SEG_CH_THREADS) void k_seg_chunk(SegArgs a) {
  using K = typename KeyTraits<KK>::K;
  constexpr int NT = SEG_CH_THREADS, CPT = SEG_CH / NT;
  // LDS position p (chunk position p - 1; halo keys at both ends) lives at
  // p + p / 32: each thread walks 32 consecutive positions, and the pad word
  // per 32 puts the 64 lanes of a wave on distinct banks
  __shared__ K s_k[SEG_CH + 2 + (SEG_CH + 2) / 32 + 1];
  auto sk = [&](uint32_t p) -> K& { return s_k[p + (p >> 5)]; };
  __shared__ int s_max[NT / WAVE];
  __shared__ double s_red[NT / WAVE];
  __shared__ uint32_t s_carry;
  const int t = threadIdx.x;
  uint32_t nch = a.chunks->ntiles_next;
  nch = nch < a.chunk_cap ? nch : a.chunk_cap;
  const uint32_t nl = a.chunks->nsegs_next;
  for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
    __syncthreads();  // the previous chunk's LDS contents are consumed
    const uint32_t li = ss_seg_of_tile(a.large, nl, c);
    const SsSeg g = a.large[li];
    const uint32_t size = g.size;
    if (a.bounds[2 * li] != 0 || a.bounds[2 * li + 1] != size) {  // holds NaNs: no features
      if (t == 0) a.partial[c] = 0.0;
      continue;
    }
    const K* __restrict__ keys = (const K*)a.kout + g.start;
    auto mapped = [&](uint32_t j) {
      K x = keys[j];
      if constexpr (key_mapped<KK>) x = map_key<KK>(x);
      return x;
    };
    const uint32_t c0 = (c - g.first_tile) * SEG_CH;
    const uint32_t cnt = size - c0 < SEG_CH ? size - c0 : SEG_CH;
    // every load of the chunk in flight at once: the segment's ends (its
    // min and max, sorted), the chunk's keys and the halo keys
    const K kmin = mapped(0), kmax = mapped(size - 1);
    K v[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const uint32_t j = (uint32_t)t + (uint32_t)q * NT;
      v[q] = j < cnt ? mapped(c0 + j) : K(0);
    }
    if (t == 0) sk(0) = c0 > 0 ? mapped(c0 - 1) : K(0);
    if (t == 1) sk(cnt + 1) = c0 + cnt < size ? mapped(c0 + cnt) : K(0);
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const uint32_t j = (uint32_t)t + (uint32_t)q * NT;
      if (j < cnt) sk(j + 1) = v[q];
    }
    uint32_t shift, nbins;
    shift_nbins((uint64_t)(kmax - kmin), shift, nbins);
    auto binof = [&](K x) { return (uint64_t)((x - kmin) >> shift); };
    __syncthreads();
    const bool carry_needed = c0 > 0 && binof(sk(0)) == binof(sk(1));
    if (carry_needed && t < WAVE) {
      // smallest position p <= c0 with bin(p) == bin(c0)
      const uint64_t target = binof(sk(1));
      int64_t R = c0;  // bin(R) == target
      int64_t step = 1, L = 0;
      for (;;) {
        const int64_t pos = R - step * (int64_t)(lane_id() + 1);
        const bool less = pos < L || binof(mapped((uint32_t)pos)) < target;
        const uint64_t m = __ballot(less);
        if (m == 0) {
          R -= step * WAVE;
          step *= WAVE;
          continue;
        }
        const int l = __builtin_ctzll(m);
        const int64_t same = R - step * l, below = R - step * (l + 1);
        if (step == 1) {
          R = same;
          break;
        }
        L = below + 1 > L ? below + 1 : L;
        R = same;
        step = (step + WAVE - 1) / WAVE;
      }
      if (t == 0) s_carry = (uint32_t)R;
    }
    __syncthreads();
    const uint32_t carry = carry_needed ? s_carry : c0;
    // bins of my positions j0 - 1 .. j0 + CPT (LDS positions j0 .. j0 + CPT
    // + 1), read once; a bin is below 65,536, so 32 bits hold it
    const uint32_t j0 = (uint32_t)t * CPT;
    uint32_t b[CPT + 2];
#pragma unroll
    for (int q = 0; q < CPT + 2; ++q) b[q] = j0 + q <= cnt + 1 ? (uint32_t)binof(sk(j0 + q)) : 0u;
    // run starts in my positions
    int last = -1;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const uint32_t j = j0 + q;
      const bool st = j < cnt && ((c0 + j == 0) || b[q] != b[q + 1]);
      if (st) last = (int)j;
    }
    int cur = block_excl_max<NT>(last, s_max);
    const double inv_n = 1.0 / (double)size;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const uint32_t j = j0 + q;
      if (j < cnt) {  // a guard, not a loop exit: the loop stays unrolled over registers
        if ((c0 + j == 0) || b[q] != b[q + 1]) cur = (int)j;
        const bool end = (c0 + j + 1 == size) || b[q + 2] != b[q + 1];
        if (end) {
          const uint32_t start = cur >= 0 ? c0 + (uint32_t)cur : carry;
          const double p = (double)(c0 + j + 1 - start) * inv_n;
          acc -= p * log2(p);
        }
      }
    }
    acc = wave_sum(acc);
    if (lane_id() == 0) s_red[t / WAVE] = acc;
    __syncthreads();
    if (t == 0) {
      double sum = 0.0;
      for (int i = 0; i < NT / WAVE; ++i) sum += s_red[i];
      a.partial[c] = sum;
    }
  }
}

// One workgroup per large segment: features from its ends and its chunks'
// entropy terms (summed in a fixed order).  The decision was taken before
// the segment was sorted.
template <int KK>
__global__ __launch_bounds__(256) void k_seg_large_final(SegArgs a) {
  using K = typename KeyTraits<KK>::K;
  __shared__ double s_red[256 / WAVE];
  const uint32_t count = a.ctr->bad ? 0u : a.ctr->nlarge;
  const int t = threadIdx.x;
  for (uint32_t i = blockIdx.x; i < count; i += gridDim.x) {
    const SsSeg g = a.large[i];
    const uint32_t s = a.large_ids[i];
    const uint32_t lo = a.bounds[2 * i], hi = a.bounds[2 * i + 1];
    const uint32_t nchunk = (g.size + SEG_CH - 1) / SEG_CH;
    double acc = 0.0;
    for (uint32_t k = t; k < nchunk; k += 256) acc += a.partial[g.first_tile + k];
    acc = wave_sum(acc);
    __syncthreads();
    if (lane_id() == 0) s_red[t / WAVE] = acc;
    __syncthreads();
    if (t != 0) continue;
    double H = 0.0;
    for (int w = 0; w < 256 / WAVE; ++w) H += s_red[w];
    DevFeatures f = {};
    f.n = g.size;
    f.nan_count = lo + (g.size - hi);
    if (!f.nan_count) {
      const K* __restrict__ keys = (const K*)a.kout + g.start;
      K mn = keys[0], mx = keys[g.size - 1];
      if constexpr (key_mapped<KK>) {
        mn = map_key<KK>(mn);
        mx = map_key<KK>(mx);
      }
      f.min_key = mn;
      f.max_key = mx;
      f.span = (uint64_t)(mx - mn);
      shift_nbins(f.span, f.shift, f.nbins);
      f.exact = f.shift == 0;
      f.entropy_bits = H < 0.0 ? 0.0 : H;
      f.entropy_ratio = f.nbins > 1 ? f.entropy_bits / log2((double)f.nbins) : 0.0;
    }
    if (a.feats) a.feats[s] = f;
  }
}

__global__ void k_seg_status(const SegCounters* __restrict__ ctr, const SsCounters* __restrict__ levels, int nlevels,
                             const SegDispatchCounters* __restrict__ dctr, uint64_t max_seg,
                             uint32_t* __restrict__ status) {
  if (threadIdx.x != 0) return;
  uint32_t st = ctr->bad ? SEG_ERR_OFFSETS : 0u;
  if (dctr && dctr->bad) st |= SEG_ERR_OVERFLOW;
  // the level count and the look-back word width were chosen for segments of
  // at most max_seg keys: a larger one is an error even if it was sorted
  if (!ctr->bad && (uint64_t)ctr->max_large > max_seg) st |= SEG_ERR_HINT;
  for (int l = 0; l < nlevels; ++l)
    if (levels[l].overflow) st |= SEG_ERR_OVERFLOW;
  if (!ctr->bad && ctr->nlarge > 0 && (nlevels == 0 || levels[nlevels - 1].nsegs_next > 0)) st |= SEG_ERR_LEVELS;
  *status = st;
}

// SplitMix64 finaliser over a counter: synthetic keys for tuning runs only.
template <int KK>
__global__ __launch_bounds__(256) void k_tune_fill(typename KeyTraits<KK>::K* __restrict__ keys, uint64_t n,
                                                   uint64_t seed) {
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    if constexpr (KK == KK_U32 || KK == KK_I32) {
      keys[i] = (uint32_t)(z >> 32);
    } else if constexpr (KK == KK_U64 || KK == KK_I64) {
      keys[i] = z;
    } else if constexpr (KK == KK_F32) {
      const float x = (float)(z >> 40) * (1.0f / 16777216.0f) * 2000.0f - 1000.0f;
      keys[i] = __float_as_uint(x);
    } else {
      const double x = (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2000.0 - 1000.0;
      keys[i] = (uint64_t)__double_as_longlong(x);
    }
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_seg_classify(const uint64_t* offs, uint32_t nseg, uint64_t n_total, uint32_t* queues, uint32_t qcap,
                               SegLarge* linfo, SsSeg* large, uint32_t* large_ids, SegCounters* ctr, hipStream_t s) {
  const uint32_t nb = (uint32_t)(((uint64_t)nseg + 256) / 256);  // nseg < 2^32: at most 2^24 workgroups of 256
  k_seg_classify<<<nb, 256, 0, s>>>(offs, nseg, n_total, queues, qcap, linfo, large, large_ids, ctr);
  return hipGetLastError();
}

hipError_t launch_seg_gate(const SegCounters* ctr, SsCounters* rec_chunks, hipStream_t s) {
  k_seg_gate<<<1, 64, 0, s>>>(ctr, rec_chunks);
  return hipGetLastError();
}

template <int KK, bool PAY>
static const void* small_fn(int variant) {
  switch (variant) {
    case 0: return reinterpret_cast<const void*>(&k_seg_small<KK, PAY, 1024, 256>);
    case 1: return reinterpret_cast<const void*>(&k_seg_small<KK, PAY, 2048, 256>);
    case 2: return reinterpret_cast<const void*>(&k_seg_small<KK, PAY, 4096, 256>);
    default: return reinterpret_cast<const void*>(&k_seg_small<KK, PAY, 8192, 512>);
  }
}

template <int KK, bool PAY>
static hipError_t small_kk(const SegArgs& a, int cls, int variant, uint32_t grid, hipStream_t s) {
  switch (variant) {
    case 0: k_seg_small<KK, PAY, 1024, 256><<<grid, 256, 0, s>>>(a, cls); break;
    case 1: k_seg_small<KK, PAY, 2048, 256><<<grid, 256, 0, s>>>(a, cls); break;
    case 2: k_seg_small<KK, PAY, 4096, 256><<<grid, 256, 0, s>>>(a, cls); break;
    case 3: k_seg_small<KK, PAY, 8192, 512><<<grid, 512, 0, s>>>(a, cls); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_seg_small(int kk, int with_vals, const SegArgs& a, int cls, int variant, uint32_t nblocks,
                            hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (nblocks > MAX_GRID_BLOCKS) nblocks = MAX_GRID_BLOCKS;  // the kernel strides over its queue
  if (cls < 0 || cls >= SEG_NCLASS || variant < cls || variant >= SEG_NVARIANT) return hipErrorInvalidValue;
  switch (kk * 2 + (with_vals ? 1 : 0)) {
    case KK_U32 * 2: return small_kk<KK_U32, false>(a, cls, variant, nblocks, s);
    case KK_U32 * 2 + 1: return small_kk<KK_U32, true>(a, cls, variant, nblocks, s);
    case KK_U64 * 2: return small_kk<KK_U64, false>(a, cls, variant, nblocks, s);
    case KK_U64 * 2 + 1: return small_kk<KK_U64, true>(a, cls, variant, nblocks, s);
    case KK_F32 * 2: return small_kk<KK_F32, false>(a, cls, variant, nblocks, s);
    case KK_I32 * 2: return small_kk<KK_I32, false>(a, cls, variant, nblocks, s);
    case KK_F32 * 2 + 1: return small_kk<KK_F32, true>(a, cls, variant, nblocks, s);
    case KK_I32 * 2 + 1: return small_kk<KK_I32, true>(a, cls, variant, nblocks, s);
    case KK_F64 * 2: return small_kk<KK_F64, false>(a, cls, variant, nblocks, s);
    case KK_I64 * 2: return small_kk<KK_I64, false>(a, cls, variant, nblocks, s);
    case KK_F64 * 2 + 1: return small_kk<KK_F64, true>(a, cls, variant, nblocks, s);
    case KK_I64 * 2 + 1: return small_kk<KK_I64, true>(a, cls, variant, nblocks, s);
    default: return hipErrorInvalidValue;
  }
}

uint32_t seg_small_resident(int kk, int with_vals, int variant, uint32_t cu_count) {
  const void* fn = nullptr;
  switch (kk * 2 + (with_vals ? 1 : 0)) {
    case KK_U32 * 2: fn = small_fn<KK_U32, false>(variant); break;
    case KK_U32 * 2 + 1: fn = small_fn<KK_U32, true>(variant); break;
    case KK_U64 * 2: fn = small_fn<KK_U64, false>(variant); break;
    case KK_U64 * 2 + 1: fn = small_fn<KK_U64, true>(variant); break;
    case KK_F32 * 2: fn = small_fn<KK_F32, false>(variant); break;
    case KK_I32 * 2: fn = small_fn<KK_I32, false>(variant); break;
    case KK_F32 * 2 + 1: fn = small_fn<KK_F32, true>(variant); break;
    case KK_I32 * 2 + 1: fn = small_fn<KK_I32, true>(variant); break;
    case KK_F64 * 2: fn = small_fn<KK_F64, false>(variant); break;
    case KK_I64 * 2: fn = small_fn<KK_I64, false>(variant); break;
    case KK_I64 * 2 + 1: fn = small_fn<KK_I64, true>(variant); break;
    default: fn = small_fn<KK_F64, true>(variant); break;
  }
  int per_cu = 0;
  const int threads = variant == 3 ? 512 : 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  return (uint32_t)per_cu * (cu_count ? cu_count : 1);
}

hipError_t launch_seg_large(int kk, const SegArgs& a, uint32_t bound_blocks, uint32_t chunk_blocks,
                            uint32_t final_blocks, hipStream_t s) {
  if (bound_blocks == 0 || chunk_blocks == 0 || final_blocks == 0) return hipSuccess;
  // every kernel here strides over its work
  bound_blocks = bound_blocks < MAX_GRID_BLOCKS ? bound_blocks : MAX_GRID_BLOCKS;
  chunk_blocks = chunk_blocks < MAX_GRID_BLOCKS ? chunk_blocks : MAX_GRID_BLOCKS;
  final_blocks = final_blocks < MAX_GRID_BLOCKS ? final_blocks : MAX_GRID_BLOCKS;
  switch (kk) {
    case KK_U32:
      k_seg_bounds<KK_U32><<<bound_blocks, 64, 0, s>>>(a);
      k_seg_chunk<KK_U32><<<chunk_blocks, SEG_CH_THREADS, 0, s>>>(a);
      k_seg_large_final<KK_U32><<<final_blocks, 256, 0, s>>>(a);
      break;
    case KK_U64:
      k_seg_bounds<KK_U64><<<bound_blocks, 64, 0, s>>>(a);
      k_seg_chunk<KK_U64><<<chunk_blocks, SEG_CH_THREADS, 0, s>>>(a);
      k_seg_large_final<KK_U64><<<final_blocks, 256, 0, s>>>(a);
      break;
    case KK_F32:
      k_seg_bounds<KK_F32><<<bound_blocks, 64, 0, s>>>(a);
      k_seg_chunk<KK_F32><<<chunk_blocks, SEG_CH_THREADS, 0, s>>>(a);
      k_seg_large_final<KK_F32><<<final_blocks, 256, 0, s>>>(a);
      break;
    case KK_F64:
      k_seg_bounds<KK_F64><<<bound_blocks, 64, 0, s>>>(a);
      k_seg_chunk<KK_F64><<<chunk_blocks, SEG_CH_THREADS, 0, s>>>(a);
      k_seg_large_final<KK_F64><<<final_blocks, 256, 0, s>>>(a);
      break;
    case KK_I32:
      k_seg_bounds<KK_I32><<<bound_blocks, 64, 0, s>>>(a);
      k_seg_chunk<KK_I32><<<chunk_blocks, SEG_CH_THREADS, 0, s>>>(a);
      k_seg_large_final<KK_I32><<<final_blocks, 256, 0, s>>>(a);
      break;
    case KK_I64:
      k_seg_bounds<KK_I64><<<bound_blocks, 64, 0, s>>>(a);
      k_seg_chunk<KK_I64><<<chunk_blocks, SEG_CH_THREADS, 0, s>>>(a);
      k_seg_large_final<KK_I64><<<final_blocks, 256, 0, s>>>(a);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

uint32_t seg_chunk_resident(int kk, uint32_t cu_count) {
  const void* fn = kk == KK_U32 ? reinterpret_cast<const void*>(&k_seg_chunk<KK_U32>)
                 : kk == KK_U64 ? reinterpret_cast<const void*>(&k_seg_chunk<KK_U64>)
                 : kk == KK_F32 ? reinterpret_cast<const void*>(&k_seg_chunk<KK_F32>)
                 : kk == KK_I32 ? reinterpret_cast<const void*>(&k_seg_chunk<KK_I32>)
                 : kk == KK_I64 ? reinterpret_cast<const void*>(&k_seg_chunk<KK_I64>)
                                : reinterpret_cast<const void*>(&k_seg_chunk<KK_F64>);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, SEG_CH_THREADS, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return (uint32_t)per_cu * (cu_count ? cu_count : 1);
}

hipError_t launch_seg_status(const SegCounters* ctr, const SsCounters* levels, int nlevels,
                             const SegDispatchCounters* dctr, uint64_t max_seg, uint32_t* status, hipStream_t s) {
  k_seg_status<<<1, 64, 0, s>>>(ctr, levels, nlevels, dctr, max_seg, status);
  return hipGetLastError();
}

hipError_t launch_tune_fill(int kk, void* keys, uint64_t n, uint64_t seed, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint64_t nb = (n + 255) / 256;
  const uint32_t grid = (uint32_t)(nb < 8192 ? nb : 8192);
  switch (kk) {
    case KK_U32: k_tune_fill<KK_U32><<<grid, 256, 0, s>>>((uint32_t*)keys, n, seed); break;
    case KK_U64: k_tune_fill<KK_U64><<<grid, 256, 0, s>>>((uint64_t*)keys, n, seed); break;
    case KK_F32: k_tune_fill<KK_F32><<<grid, 256, 0, s>>>((uint32_t*)keys, n, seed); break;
    case KK_I32: k_tune_fill<KK_I32><<<grid, 256, 0, s>>>((uint32_t*)keys, n, seed); break;
    case KK_F64: k_tune_fill<KK_F64><<<grid, 256, 0, s>>>((uint64_t*)keys, n, seed); break;
    case KK_I64: k_tune_fill<KK_I64><<<grid, 256, 0, s>>>((uint64_t*)keys, n, seed); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ahs
