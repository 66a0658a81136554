// Feature extraction on gfx950 (Sec. III-A): min/max over mapped keys with
// a NaN count, the binned key histogram and its Shannon entropy in FP64.
//
// Bins: (key - min) >> shift with the smallest shift giving at most 65,536
// bins.  Up to 8,192 bins (span < 8,192, always exact) the histogram lives
// in LDS as u32 counters; above that as 65,536 packed u16 counters (128 KiB)
// whose 16-bit overflows are detected from the atomic's return value and
// carried exactly into a global correction array.
#include "histcommon.hpp"

namespace ahs {

// ------------------------------------------------------------------ min/max
// MOD: also counts each non-NaN key by its mapped value modulo
// HIST_SMALL_MAX_BINS (a speculative histogram: exact, up to a rotation by
// min, whenever the span is below HIST_SMALL_MAX_BINS) into
// mod_part[block][.]; NaN keys go to a spare counter.
template <int KK, bool MOD>
__global__ __launch_bounds__(MINMAX_THREADS) void k_minmax(const typename KeyTraits<KK>::K* __restrict__ keys,
                                                           uint64_t n, MinMaxPartial* __restrict__ part,
                                                           uint32_t* __restrict__ mod_part) {
  using K = typename KeyTraits<KK>::K;
  constexpr int V = 16 / sizeof(K);
  constexpr uint32_t M = HIST_SMALL_MAX_BINS;
  static_assert((M & (M - 1)) == 0, "modulo by masking");
  __shared__ uint32_t h[MOD ? M + 1 : 1];
  if constexpr (MOD) {
    for (uint32_t b = threadIdx.x; b <= M; b += MINMAX_THREADS) h[b] = 0;
    __syncthreads();
  }
  K mn = ~K(0), mx = K(0);
  uint32_t nan = 0;
  const uint64_t tid = (uint64_t)blockIdx.x * MINMAX_THREADS + threadIdx.x;
  for_each_group<K, 4>(keys, n, tid, (uint64_t)gridDim.x * MINMAX_THREADS, [&](const K (&kb)[V], int m) {
    uint32_t bins[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      bins[i] = M;
      if (i < m) {
        const K b = kb[i];
        if (KeyTraits<KK>::FLT && fnan(b)) {
          ++nan;
        } else {
          const K x = map_key<KK>(b);
          mn = x < mn ? x : mn;
          mx = x > mx ? x : mx;
          bins[i] = (uint32_t)x & (M - 1u);
        }
      }
    }
    if constexpr (MOD) lds_count_group<V>(h, bins, m);
  });
  if constexpr (MOD) {
    __syncthreads();
    uint32_t* out = mod_part + (size_t)blockIdx.x * M;
    for (uint32_t b = threadIdx.x; b < M; b += MINMAX_THREADS) out[b] = h[b];
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  nan = wave_sum(nan);
  __shared__ K smn[MINMAX_THREADS / WAVE], smx[MINMAX_THREADS / WAVE];
  __shared__ uint32_t snan[MINMAX_THREADS / WAVE];
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) { smn[w] = mn; smx[w] = mx; snan[w] = nan; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < MINMAX_THREADS / WAVE; ++i) {
      mn = smn[i] < mn ? smn[i] : mn;
      mx = smx[i] > mx ? smx[i] : mx;
      nan += snan[i];
    }
    part[blockIdx.x].mn = mn;
    part[blockIdx.x].mx = mx;
    part[blockIdx.x].nan = nan;
  }
}

// One workgroup folds the partials and derives span, shift and nbins.  With
// corr set, a plan for the packed histogram also zeroes its 65,536
// correction words here (the histogram kernel adds to them), which saves a
// fill launch.
__global__ __launch_bounds__(256) void k_minmax_final(const MinMaxPartial* __restrict__ part, int nparts,
                                                      uint64_t n, DevFeatures* __restrict__ df, FeaturePlanCfg pc,
                                                      uint32_t* __restrict__ corr) {
  __shared__ uint32_t s_plan;
  uint64_t mn = ~0ull, mx = 0, nan = 0;
  for (int i = threadIdx.x; i < nparts; i += 256) {
    mn = part[i].mn < mn ? part[i].mn : mn;
    mx = part[i].mx > mx ? part[i].mx : mx;
    nan += part[i].nan;
  }
  mn = wave_min(mn);
  mx = wave_max(mx);
  nan = wave_sum(nan);
  __shared__ uint64_t s[3][4];
  const int w = threadIdx.x / WAVE;
  if (lane_id() == 0) { s[0][w] = mn; s[1][w] = mx; s[2][w] = nan; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i) {
      mn = s[0][i] < mn ? s[0][i] : mn;
      mx = s[1][i] > mx ? s[1][i] : mx;
      nan += s[2][i];
    }
    DevFeatures f = {};
    f.n = n;
    f.nan_count = nan;
    if (nan == n) { mn = 0; mx = 0; }
    f.min_key = mn;
    f.max_key = mx;
    f.span = mx - mn;
    const int bl = bitlen64(f.span);
    f.shift = bl > 16 ? (uint32_t)(bl - 16) : 0u;
    f.nbins = (uint32_t)(f.span >> f.shift) + 1u;
    f.exact = f.shift == 0 ? 1u : 0u;
    if (pc.enabled) {
      // what the AUTO decision will need: the exact histogram when counting
      // may follow (it doubles as the counting histogram), the entropy and
      // fused digit counts when radix may follow, the entropy for the model
      const bool small_n = n <= pc.n_small;
      const bool counting = !small_n && f.span <= pc.kcount_minus1 && f.span <= 65535u;
      const bool radix = !small_n && f.span > pc.kcount_minus1 && (f.span >= pc.k_radix || pc.model);
      const bool need = n > 0 && nan == 0 && (pc.want_hist || counting || radix || (pc.model && !small_n));
      const int ndig = radix ? (bl + 7) / 8 > 1 ? (bl + 7) / 8 : 1 : 0;
      uint32_t plan = PLAN_ON | (need ? 0u : PLAN_SKIP) | ((uint32_t)ndig << 4);
      if (f.nbins > (uint32_t)HIST_SMALL_MAX_BINS || ndig > 0) plan |= PLAN_LARGE;
      // the min/max pass's modulo counts are the exact histogram when every
      // key - min lies below the modulus (shift 0, at most that many bins)
      if (pc.fused && need && !(plan & PLAN_LARGE) && f.span < (uint64_t)HIST_SMALL_MAX_BINS) plan |= PLAN_FUSED;
      f.reserved = plan;
    }
    *df = f;
    s_plan = f.reserved;
  }
  if (corr) {
    __syncthreads();
    if (s_plan & PLAN_LARGE) {
      u32x4* c4 = reinterpret_cast<u32x4*>(corr);
      const u32x4 z = {0u, 0u, 0u, 0u};
      for (int i = threadIdx.x; i < 65536 / 4; i += 256) c4[i] = z;
    }
  }
}

template <int KK>
static void minmax_kk(const void* keys, uint64_t n, MinMaxPartial* partials, int nblocks, uint32_t* mod,
                      hipStream_t s) {
  using K = typename KeyTraits<KK>::K;
  if (mod)
    k_minmax<KK, true><<<nblocks, MINMAX_THREADS, 0, s>>>((const K*)keys, n, partials, mod);
  else
    k_minmax<KK, false><<<nblocks, MINMAX_THREADS, 0, s>>>((const K*)keys, n, partials, nullptr);
}

hipError_t launch_minmax(int kk, const void* keys, uint64_t n, MinMaxPartial* partials, int nblocks,
                         DevFeatures* df, hipStream_t s, const FeaturePlanCfg* plan_cfg, uint32_t* mod_partials,
                         uint32_t* corr) {
  if (corr && !plan_cfg) return hipErrorInvalidValue;  // only a plan says whether the packed histogram follows
  switch (kk) {
    case KK_U32: minmax_kk<KK_U32>(keys, n, partials, nblocks, mod_partials, s); break;
    case KK_U64: minmax_kk<KK_U64>(keys, n, partials, nblocks, mod_partials, s); break;
    case KK_F32: minmax_kk<KK_F32>(keys, n, partials, nblocks, mod_partials, s); break;
    case KK_I32: minmax_kk<KK_I32>(keys, n, partials, nblocks, mod_partials, s); break;
    case KK_F64: minmax_kk<KK_F64>(keys, n, partials, nblocks, mod_partials, s); break;
    case KK_I64: minmax_kk<KK_I64>(keys, n, partials, nblocks, mod_partials, s); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  FeaturePlanCfg pc = {};
  if (plan_cfg) pc = *plan_cfg;
  pc.fused = (plan_cfg && mod_partials) ? 1u : 0u;
  k_minmax_final<<<1, 256, 0, s>>>(partials, nblocks, n, df, pc, corr);
  return hipGetLastError();
}

// ------------------------------------------------------------------ histograms
// Exact small histogram: nbins <= 8,192 u32 counters in LDS; each block
// writes its counts to partials[block][nbins].
template <int KK>
__global__ __launch_bounds__(HIST_SMALL_THREADS) void k_hist_small(const typename KeyTraits<KK>::K* __restrict__ keys,
                                                                   uint64_t n, typename KeyTraits<KK>::K kmin,
                                                                   uint32_t shift, uint32_t nbins,
                                                                   uint32_t* __restrict__ partials,
                                                                   const DevFeatures* __restrict__ plan) {
  using K = typename KeyTraits<KK>::K;
  __shared__ uint32_t h[HIST_SMALL_MAX_BINS];
  if (plan) {
    if (plan->reserved & (PLAN_SKIP | PLAN_LARGE | PLAN_FUSED)) return;
    kmin = (K)plan->min_key;
    shift = plan->shift;
    nbins = plan->nbins;
  }
  for (uint32_t b = threadIdx.x; b < nbins; b += HIST_SMALL_THREADS) h[b] = 0;
  __syncthreads();
  const uint64_t tid = (uint64_t)blockIdx.x * HIST_SMALL_THREADS + threadIdx.x;
  constexpr int V = 16 / sizeof(K);
  for_each_group<K, 4>(keys, n, tid, (uint64_t)gridDim.x * HIST_SMALL_THREADS, [&](const K (&kb)[V], int m) {
    uint32_t bins[V];
#pragma unroll
    for (int i = 0; i < V; ++i) bins[i] = (uint32_t)((map_key<KK>(kb[i]) - kmin) >> shift);
    lds_count_group<V>(h, bins, m);
  });
  __syncthreads();
  uint32_t* out = partials + (size_t)blockIdx.x * nbins;
  for (uint32_t b = threadIdx.x; b < nbins; b += HIST_SMALL_THREADS) out[b] = h[b];
}

hipError_t launch_hist_small(int kk, const void* keys, uint64_t n, uint64_t kmin, uint32_t shift,
                             uint32_t nbins, uint32_t* partials, int nblocks, hipStream_t s, const DevFeatures* plan) {
  if (!plan && nbins > (uint32_t)HIST_SMALL_MAX_BINS) return hipErrorInvalidValue;
  switch (kk) {
    case KK_U32: k_hist_small<KK_U32><<<nblocks, HIST_SMALL_THREADS, 0, s>>>((const uint32_t*)keys, n, (uint32_t)kmin, shift, nbins, partials, plan); break;
    case KK_U64: k_hist_small<KK_U64><<<nblocks, HIST_SMALL_THREADS, 0, s>>>((const uint64_t*)keys, n, kmin, shift, nbins, partials, plan); break;
    case KK_F32: k_hist_small<KK_F32><<<nblocks, HIST_SMALL_THREADS, 0, s>>>((const uint32_t*)keys, n, (uint32_t)kmin, shift, nbins, partials, plan); break;
    case KK_I32: k_hist_small<KK_I32><<<nblocks, HIST_SMALL_THREADS, 0, s>>>((const uint32_t*)keys, n, (uint32_t)kmin, shift, nbins, partials, plan); break;
    case KK_F64: k_hist_small<KK_F64><<<nblocks, HIST_SMALL_THREADS, 0, s>>>((const uint64_t*)keys, n, kmin, shift, nbins, partials, plan); break;
    case KK_I64: k_hist_small<KK_I64><<<nblocks, HIST_SMALL_THREADS, 0, s>>>((const uint64_t*)keys, n, kmin, shift, nbins, partials, plan); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Large histogram: 65,536 bins as packed u16 pairs in 128 KiB of LDS.  Word
// w holds bin 2w in its low half and bin 2w+1 in its high half.  All counter
// arithmetic is additive modulo 2^32, so overflows are repaired exactly:
//   low half wraps (old low == 0xFFFF): bin 2w gets +65,536 and the carry
//     that leaked into the high half is taken back (bin 2w+1 gets -1); if the
//     whole word wrapped (old == 0xFFFFFFFF) that carry also left the word,
//     so bin 2w+1 gets +65,536 as well;
//   high half wraps (old high == 0xFFFF): bin 2w+1 gets +65,536.
// The final count of bin b is sum over blocks of its half plus corr[b],
// modulo 2^32, which is exact because every true count is below 2^32.
// Optionally also counts ndig 8-bit digits of (key - min) per key: the
// upfront digit histogram of the LSD radix sort, fused into the same read.
template <int KK, bool DIG>
__global__ __launch_bounds__(HIST_LARGE_THREADS) void k_hist_large(const typename KeyTraits<KK>::K* __restrict__ keys,
                                                                   uint64_t n, typename KeyTraits<KK>::K kmin,
                                                                   uint32_t shift, uint32_t* __restrict__ partials,
                                                                   uint32_t* __restrict__ corr, int ndig,
                                                                   uint32_t* __restrict__ digit_partials,
                                                                   const DevFeatures* __restrict__ plan) {
  using K = typename KeyTraits<KK>::K;
  constexpr int V = 16 / sizeof(K);  // keys per 16-byte load
  // digit counters: DCOPY copies, lane l counting into copy l % DCOPY, so
  // that lanes holding one frequent key (skewed input) hit DCOPY different
  // addresses; copies are offset by 16 banks
  constexpr int DMAX = sizeof(K);  // 8-bit digits of a key
  constexpr int DCOPY = DIG ? (sizeof(K) == 4 ? AHS_DIG_COPIES32 : AHS_DIG_COPIES64) : 1;
  constexpr int DSTRIDE = DMAX * 256 + 16;
  __shared__ uint32_t h[HIST_LARGE_WORDS];
  __shared__ uint32_t dh[DIG ? DCOPY * DSTRIDE : 1];
  static_assert(sizeof(h) + sizeof(dh) <= 160 * 1024, "LDS");
  if (plan) {
    const uint32_t p = plan->reserved;
    if (p & PLAN_SKIP) return;
    kmin = (K)plan->min_key;
    shift = plan->shift;
    if (!(p & PLAN_LARGE)) {
      // the exact histogram of at most HIST_SMALL_MAX_BINS bins, unless the
      // min/max pass already counted it: plain counters in the first words
      // of the LDS array, one row of nbins per workgroup
      if (p & PLAN_FUSED) return;
      const uint32_t nbins = plan->nbins;
      for (uint32_t b = threadIdx.x; b < nbins; b += HIST_LARGE_THREADS) h[b] = 0;
      __syncthreads();
      const uint64_t tid = (uint64_t)blockIdx.x * HIST_LARGE_THREADS + threadIdx.x;
      for_each_group<K, 4>(keys, n, tid, (uint64_t)gridDim.x * HIST_LARGE_THREADS, [&](const K (&kb)[V], int m) {
        uint32_t bins[V];
#pragma unroll
        for (int i = 0; i < V; ++i) bins[i] = (uint32_t)((map_key<KK>(kb[i]) - kmin) >> shift);
        lds_count_group<V>(h, bins, m);
      });
      __syncthreads();
      uint32_t* out = partials + (size_t)blockIdx.x * nbins;
      for (uint32_t b = threadIdx.x; b < nbins; b += HIST_LARGE_THREADS) out[b] = h[b];
      return;
    }
    ndig = DIG ? plan_fused_digits(p, shift) : 0;
  }
  ndig = ndig < DMAX ? ndig : DMAX;  // the counters hold one key's digits
  for (int i = threadIdx.x; i < HIST_LARGE_WORDS; i += HIST_LARGE_THREADS) h[i] = 0;
  if constexpr (DIG)
    for (int i = threadIdx.x; i < DCOPY * DSTRIDE; i += HIST_LARGE_THREADS) dh[i] = 0;
  __syncthreads();
  uint32_t* const mydh = dh + (DIG ? (lane_id() % DCOPY) * DSTRIDE : 0);

  // Repairs a 16-bit wrap after c was added to bin `bin`, whose word held
  // `old` before the add.
  auto fix_packed = [&](uint32_t bin, uint32_t old, uint32_t c) {
    if (bin & 1u) {
      if ((old >> 16) + c > 0xFFFFu) add_agent(&corr[bin], 65536u);
    } else if ((old & 0xFFFFu) + c > 0xFFFFu) {
      add_agent(&corr[bin], 65536u);
      add_agent(&corr[bin + 1], (old >> 16) == 0xFFFFu ? 65535u : 0xFFFFFFFFu);
    }
  };
  auto packed_add = [&](uint32_t bin, uint32_t c) {
    return atomicAdd(&h[bin >> 1], (bin & 1u) ? (c << 16) : c);
  };

  const uint64_t nthreads = (uint64_t)gridDim.x * HIST_LARGE_THREADS;
  const uint64_t tid = (uint64_t)blockIdx.x * HIST_LARGE_THREADS + threadIdx.x;
  for_each_group<K, 4>(keys, n, tid, nthreads, [&](const K (&kb)[V], int m) {
    K off[V];
    uint32_t bins[V];
    bool pend[V];
#pragma unroll
    for (int i = 0; i < V; ++i) {
      off[i] = map_key<KK>(kb[i]) - kmin;
      bins[i] = (uint32_t)(off[i] >> shift);
      pend[i] = i < m;
    }
    // a dominant bin of the wave through one lane; every other key with its
    // own atomic: independent returning atomics first, overflow repairs after
    const uint32_t c = __builtin_amdgcn_readfirstlane(bins[0]);
    if (wave_bin_dominant<V>(bins, c)) {
      const uint32_t hit = take_wave_bin<V>(bins, pend, c);
      if (mbcnt(__ballot(1)) == 0) fix_packed(c, packed_add(c, hit), hit);
    }
    uint32_t olds[V];
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (pend[i]) olds[i] = packed_add(bins[i], 1u);
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (pend[i]) fix_packed(bins[i], olds[i], 1u);
    if constexpr (DIG) {
      for (int p = 0; p < ndig; ++p) {
        uint32_t dg[V];
#pragma unroll
        for (int i = 0; i < V; ++i) dg[i] = (uint32_t)((off[i] >> (8 * p)) & 255u);
        lds_count_group<V>(mydh + p * 256, dg, m);
      }
    }
  });
  __syncthreads();
  uint32_t* out = partials + (size_t)blockIdx.x * HIST_LARGE_WORDS;
  for (int i = threadIdx.x; i < HIST_LARGE_WORDS; i += HIST_LARGE_THREADS) out[i] = h[i];
  if constexpr (DIG) {
    uint32_t* dout = digit_partials + (size_t)blockIdx.x * ndig * 256;
    for (int i = threadIdx.x; i < ndig * 256; i += HIST_LARGE_THREADS) {
      uint32_t t = 0;
#pragma unroll
      for (int r = 0; r < DCOPY; ++r) t += dh[r * DSTRIDE + i];
      dout[i] = t;
    }
  }
}

template <int KK>
static hipError_t hist_large_kk(const void* keys, uint64_t n, uint64_t kmin, uint32_t shift, uint32_t* partials,
                                uint32_t* corr, int nblocks, int ndig, uint32_t* dparts, hipStream_t s,
                                const DevFeatures* plan) {
  using K = typename KeyTraits<KK>::K;
  if (ndig > 0 || plan)  // with a plan the digit count is read on the device
    k_hist_large<KK, true><<<nblocks, HIST_LARGE_THREADS, 0, s>>>((const K*)keys, n, (K)kmin, shift, partials, corr, ndig, dparts, plan);
  else
    k_hist_large<KK, false><<<nblocks, HIST_LARGE_THREADS, 0, s>>>((const K*)keys, n, (K)kmin, shift, partials, corr, 0, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_hist_large(int kk, const void* keys, uint64_t n, uint64_t kmin, uint32_t shift,
                             uint32_t* partials, uint32_t* corr, int nblocks, int ndig,
                             uint32_t* digit_partials, hipStream_t s, const DevFeatures* plan) {
  if (ndig < 0 || ndig > key_bytes_of(kk)) return hipErrorInvalidValue;
  switch (kk) {
    case KK_U32: return hist_large_kk<KK_U32>(keys, n, kmin, shift, partials, corr, nblocks, ndig, digit_partials, s, plan);
    case KK_U64: return hist_large_kk<KK_U64>(keys, n, kmin, shift, partials, corr, nblocks, ndig, digit_partials, s, plan);
    case KK_F32: return hist_large_kk<KK_F32>(keys, n, kmin, shift, partials, corr, nblocks, ndig, digit_partials, s, plan);
    case KK_I32: return hist_large_kk<KK_I32>(keys, n, kmin, shift, partials, corr, nblocks, ndig, digit_partials, s, plan);
    case KK_F64: return hist_large_kk<KK_F64>(keys, n, kmin, shift, partials, corr, nblocks, ndig, digit_partials, s, plan);
    case KK_I64: return hist_large_kk<KK_I64>(keys, n, kmin, shift, partials, corr, nblocks, ndig, digit_partials, s, plan);
    default: return hipErrorInvalidValue;
  }
}

// Folds the per-block histograms into the final counts, writes them (when
// hist_out is non-null) and sums the entropy terms -(c/n) log2(c/n) of the
// block's bins in FP64 into hpart[block].  Each block covers HRED_ITEMS
// items (packed words for large histograms, bins for small ones) with
// HRED_SLICES threads per item splitting the per-block partials.
constexpr int HRED_THREADS = 256;
constexpr int HRED_SLICES = 8;
constexpr int HRED_ITEMS = HRED_THREADS / HRED_SLICES;

__global__ __launch_bounds__(HRED_THREADS) void k_hist_reduce(const uint32_t* __restrict__ partials, int ngroups,
                                                              uint32_t nbins, int large,
                                                              const uint32_t* __restrict__ corr,
                                                              uint32_t* __restrict__ hist_out, uint64_t n,
                                                              double* __restrict__ hpart,
                                                              const DevFeatures* __restrict__ plan,
                                                              int ngroups_large, int ngroups_fused) {
  __shared__ uint32_t s0[HRED_SLICES][HRED_ITEMS], s1[HRED_SLICES][HRED_ITEMS];
  const int it = threadIdx.x % HRED_ITEMS, sl = threadIdx.x / HRED_ITEMS;
  if (plan) {
    const uint32_t p = plan->reserved;
    if (p & PLAN_SKIP) {
      if (threadIdx.x == 0) hpart[blockIdx.x] = 0.0;
      return;
    }
    large = (p & PLAN_LARGE) ? 1 : 0;
    nbins = plan->nbins;
    if (large) ngroups = ngroups_large;
    if (p & PLAN_FUSED) ngroups = ngroups_fused;
  }
  // fused: block g's count of key - min == b sits at its modulo slot (b + min) mod M
  const bool fused = plan && (plan->reserved & PLAN_FUSED);
  const uint32_t rot = fused ? (uint32_t)plan->min_key & (uint32_t)(HIST_SMALL_MAX_BINS - 1) : 0u;
  const uint32_t item = blockIdx.x * HRED_ITEMS + it;
  const uint32_t nitems = large ? (nbins + 1u) / 2u : nbins;
  uint32_t c0 = 0, c1 = 0;
  if (item < nitems) {
    if (large) {
      for (int g = sl; g < ngroups; g += HRED_SLICES) {
        const uint32_t w = partials[(size_t)g * HIST_LARGE_WORDS + item];
        c0 += w & 0xFFFFu;
        c1 += w >> 16;
      }
    } else if (fused) {
      const uint32_t slot = (item + rot) & (uint32_t)(HIST_SMALL_MAX_BINS - 1);
      for (int g = sl; g < ngroups; g += HRED_SLICES) c0 += partials[(size_t)g * HIST_SMALL_MAX_BINS + slot];
    } else {
      for (int g = sl; g < ngroups; g += HRED_SLICES) c0 += partials[(size_t)g * nbins + item];
    }
  }
  s0[sl][it] = c0;
  s1[sl][it] = c1;
  __syncthreads();
  const double inv_n = 1.0 / (double)n;
  double term = 0.0;
  if (sl == 0 && item < nitems) {
    for (int q = 1; q < HRED_SLICES; ++q) {
      c0 += s0[q][it];
      c1 += s1[q][it];
    }
    if (large) {
      c0 += corr[2 * item];
      c1 += corr[2 * item + 1];
      if (hist_out) {
        hist_out[2 * item] = c0;
        if (2 * item + 1 < nbins) hist_out[2 * item + 1] = c1;
      }
      if (c0) { const double p = (double)c0 * inv_n; term -= p * log2(p); }
      if (2 * item + 1 < nbins && c1) { const double p = (double)c1 * inv_n; term -= p * log2(p); }
    } else {
      if (hist_out) hist_out[item] = c0;
      if (c0) { const double p = (double)c0 * inv_n; term -= p * log2(p); }
    }
  }
  term = wave_sum(term);
  __shared__ double s[HRED_THREADS / WAVE];
  if (lane_id() == 0) s[threadIdx.x / WAVE] = term;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int i = 0; i < HRED_THREADS / WAVE; ++i) acc += s[i];
    hpart[blockIdx.x] = acc;
  }
}

hipError_t launch_hist_reduce(const uint32_t* partials, int ngroups, uint32_t nbins, int large,
                              const uint32_t* corr, uint32_t* hist_out, uint64_t n, double* hpart,
                              int* nparts_out, hipStream_t s, const DevFeatures* plan, int ngroups_large,
                              int ngroups_fused) {
  const uint32_t items = large ? (nbins + 1u) / 2u : nbins;
  // with a plan the bins are known on the device only: cover the largest
  // histogram; blocks past the last bin contribute a zero partial
  const int nb = plan ? HRED_MAX_BLOCKS : (int)((items + HRED_ITEMS - 1) / HRED_ITEMS);
  *nparts_out = nb;
  k_hist_reduce<<<nb, HRED_THREADS, 0, s>>>(partials, ngroups, nbins, large, corr, hist_out, n, hpart, plan,
                                            ngroups_large, ngroups_fused);
  return hipGetLastError();
}

// Sums the per-block entropy partials in a fixed order (256 strided sums,
// then those in order) and sets the ratio.  Threads 0..255 of the workgroup
// do the work; every thread of it must call this (it holds a barrier).
__device__ __forceinline__ void entropy_final_block(const double* __restrict__ hpart, int nparts,
                                                    DevFeatures* df, double* s) {
  if (threadIdx.x < 256) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += hpart[i];
    s[threadIdx.x] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double H = 0.0;
    for (int i = 0; i < 256; ++i) H += s[i];
    if (H < 0.0) H = 0.0;
    df->entropy_bits = H;
    df->entropy_ratio = df->nbins > 1 ? H / log2((double)df->nbins) : 0.0;
  }
}

__global__ __launch_bounds__(256) void k_entropy_final(const double* __restrict__ hpart, int nparts,
                                                       DevFeatures* __restrict__ df) {
  __shared__ double s[256];
  entropy_final_block(hpart, nparts, df, s);
}

hipError_t launch_entropy_final(const double* hpart, int nparts, DevFeatures* df, hipStream_t s) {
  k_entropy_final<<<1, 256, 0, s>>>(hpart, nparts, df);
  return hipGetLastError();
}

// ------------------------------------------------------------------ upfront digit counts
// Counts the ndig 8-bit digits of (key - min) of every key in one read: the
// per-pass digit histograms of the LSD radix sort.
template <int KK>
__global__ __launch_bounds__(DIGIT_HIST_THREADS) void k_digit_hist(const typename KeyTraits<KK>::K* __restrict__ keys,
                                                                   uint64_t n, typename KeyTraits<KK>::K kmin, int ndig,
                                                                   uint32_t* __restrict__ digit_partials) {
  using K = typename KeyTraits<KK>::K;
  // copies of the counters as in the fused histogram: lane l counts into
  // copy l % DCOPY
  constexpr int DCOPY = sizeof(K) == 4 ? AHS_DIG_COPIES32 : AHS_DIG_COPIES64;
  constexpr int DSTRIDE = (int)sizeof(K) * 256 + 16;
  __shared__ uint32_t dh[DCOPY * DSTRIDE];
  for (int i = threadIdx.x; i < DCOPY * DSTRIDE; i += DIGIT_HIST_THREADS) dh[i] = 0;
  __syncthreads();
  uint32_t* const mydh = dh + (lane_id() % DCOPY) * DSTRIDE;
  ndig = ndig < (int)sizeof(K) ? ndig : (int)sizeof(K);  // the counters hold one key's digits
  const uint64_t tid = (uint64_t)blockIdx.x * DIGIT_HIST_THREADS + threadIdx.x;
  constexpr int V = 16 / sizeof(K);
  for_each_group<K, 4>(keys, n, tid, (uint64_t)gridDim.x * DIGIT_HIST_THREADS, [&](const K (&kb)[V], int m) {
    K off[V];
#pragma unroll
    for (int i = 0; i < V; ++i) off[i] = map_key<KK>(kb[i]) - kmin;
    for (int p = 0; p < ndig; ++p) {
      uint32_t dg[V];
#pragma unroll
      for (int i = 0; i < V; ++i) dg[i] = (uint32_t)((off[i] >> (8 * p)) & 255u);
      lds_count_group<V>(mydh + p * 256, dg, m);
    }
  });
  __syncthreads();
  uint32_t* out = digit_partials + (size_t)blockIdx.x * ndig * 256;
  for (int i = threadIdx.x; i < ndig * 256; i += DIGIT_HIST_THREADS) {
    uint32_t t = 0;
#pragma unroll
    for (int r = 0; r < DCOPY; ++r) t += dh[r * DSTRIDE + i];
    out[i] = t;
  }
}

hipError_t launch_digit_hist(int kk, const void* keys, uint64_t n, uint64_t kmin, int ndig,
                             uint32_t* digit_partials, int nblocks, hipStream_t s) {
  if (ndig < 1 || ndig > key_bytes_of(kk)) return hipErrorInvalidValue;
  switch (kk) {
    case KK_U32: k_digit_hist<KK_U32><<<nblocks, DIGIT_HIST_THREADS, 0, s>>>((const uint32_t*)keys, n, (uint32_t)kmin, ndig, digit_partials); break;
    case KK_U64: k_digit_hist<KK_U64><<<nblocks, DIGIT_HIST_THREADS, 0, s>>>((const uint64_t*)keys, n, kmin, ndig, digit_partials); break;
    case KK_F32: k_digit_hist<KK_F32><<<nblocks, DIGIT_HIST_THREADS, 0, s>>>((const uint32_t*)keys, n, (uint32_t)kmin, ndig, digit_partials); break;
    case KK_I32: k_digit_hist<KK_I32><<<nblocks, DIGIT_HIST_THREADS, 0, s>>>((const uint32_t*)keys, n, (uint32_t)kmin, ndig, digit_partials); break;
    case KK_F64: k_digit_hist<KK_F64><<<nblocks, DIGIT_HIST_THREADS, 0, s>>>((const uint64_t*)keys, n, kmin, ndig, digit_partials); break;
    case KK_I64: k_digit_hist<KK_I64><<<nblocks, DIGIT_HIST_THREADS, 0, s>>>((const uint64_t*)keys, n, kmin, ndig, digit_partials); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Counts of one radix digit summed from the reduced 65,536-bin histogram,
// for a digit whose bits lie at q = 8p - shift >= 0 inside the bin: bins
// come in runs of 2^q sharing the digit (run index) & 255.  Pieces of L
// bins (a whole run when q <= 6, else 64 bins of one run) are summed in
// registers, each lane taking 64 / L pieces with all its loads in flight;
// lanes take consecutive pieces, so with L = 2^q the digits of a wave's
// atomics are distinct.  The histogram buffer holds 65,536 counts: loads
// past nbins stay inside it and are masked.
template <int L>
__device__ __forceinline__ void derived_digit_pieces(const uint32_t* __restrict__ hist, uint32_t nb, int q,
                                                     uint32_t* __restrict__ cnt, int t) {
  constexpr int NT = 1024;
  constexpr int PIECES = 64 / L;  // 65,536 bins / NT threads / L
  uint32_t acc[PIECES];
  if constexpr (L >= 4) {
    u32x4 w[PIECES][L / 4];
#pragma unroll
    for (int u = 0; u < PIECES; ++u) {
      const u32x4* hv = reinterpret_cast<const u32x4*>(hist + (size_t)(t + u * NT) * L);
#pragma unroll
      for (int k = 0; k < L / 4; ++k) w[u][k] = hv[k];
    }
#pragma unroll
    for (int u = 0; u < PIECES; ++u) {
      const uint32_t b0 = (uint32_t)(t + u * NT) * L;
      uint32_t a = 0;
#pragma unroll
      for (int k = 0; k < L / 4; ++k) {
        const uint32_t b = b0 + 4 * k;
        a += (b < nb ? w[u][k].x : 0u) + (b + 1 < nb ? w[u][k].y : 0u) + (b + 2 < nb ? w[u][k].z : 0u) +
             (b + 3 < nb ? w[u][k].w : 0u);
      }
      acc[u] = a;
    }
  } else {
    uint32_t v[PIECES][L];
#pragma unroll
    for (int u = 0; u < PIECES; ++u)
#pragma unroll
      for (int k = 0; k < L; ++k) v[u][k] = hist[(uint32_t)(t + u * NT) * L + k];
#pragma unroll
    for (int u = 0; u < PIECES; ++u) {
      const uint32_t b0 = (uint32_t)(t + u * NT) * L;
      uint32_t a = 0;
#pragma unroll
      for (int k = 0; k < L; ++k) a += b0 + k < nb ? v[u][k] : 0u;
      acc[u] = a;
    }
  }
#pragma unroll
  for (int u = 0; u < PIECES; ++u)
    if (acc[u]) atomicAdd(&cnt[(((uint32_t)(t + u * NT) * L) >> q) & 255u], acc[u]);
}

// One workgroup per pass.  A digit counted per key: four groups of 256
// threads (one per digit) sum interleaved quarters of the block partials
// with many loads in flight and are folded in LDS.  With a plan, a digit at
// or above the histogram's shift is summed from the reduced histogram
// instead (its value is a function of the bin; a wave whose 64 bins share
// the digit adds once).  The pass's 256 counts are then exclusively scanned.
// With hpart set, workgroup 0 first finishes the entropy into df (the
// feature vector the plan lives in), saving the launch of k_entropy_final.
constexpr int DIGIT_REDUCE_THREADS = 1024;
static_assert(DIGIT_REDUCE_THREADS * 64 == 65536, "derived digits: 64 bins per thread");
__global__ __launch_bounds__(DIGIT_REDUCE_THREADS) void k_digit_reduce(const uint32_t* __restrict__ parts,
                                                                       const uint32_t* __restrict__ hist,
                                                                       int nblocks, int ndig,
                                                                       uint32_t* __restrict__ counts,
                                                                       uint32_t* __restrict__ offsets,
                                                                       const DevFeatures* plan,
                                                                       const double* __restrict__ hpart, int nparts,
                                                                       DevFeatures* df) {
  constexpr int G = DIGIT_REDUCE_THREADS / 256;
  const int p = blockIdx.x, t = threadIdx.x, d = t % 256, g = t / 256;
  if (hpart && p == 0) {  // uniform over the workgroup
    __shared__ double s_ent[256];
    entropy_final_block(hpart, nparts, df, s_ent);
  }
  int nf = ndig;  // digits the block partials hold
  if (plan) {
    if (plan->reserved & PLAN_SKIP) return;
    ndig = plan_digits(plan->reserved);
    nf = plan_fused_digits(plan->reserved, plan->shift);
  }
  if (p >= ndig) return;  // uniform over the workgroup
  __shared__ uint32_t s_grp[G][256];
  __shared__ uint32_t s_scan[DIGIT_REDUCE_THREADS / WAVE + 1];
  uint32_t c = 0;
  if (p < nf) {
#pragma unroll 16
    for (int b = g; b < nblocks; b += G) c += parts[((size_t)b * nf + p) * 256 + d];
    s_grp[g][d] = c;
  } else {
    s_grp[g][d] = 0;
    __syncthreads();
    const int q = 8 * p - (int)plan->shift;  // 0 <= q <= 15: digit bits lie within the bin
    switch (q < 6 ? q : 6) {
      case 0: derived_digit_pieces<1>(hist, plan->nbins, q, s_grp[0], t); break;
      case 1: derived_digit_pieces<2>(hist, plan->nbins, q, s_grp[0], t); break;
      case 2: derived_digit_pieces<4>(hist, plan->nbins, q, s_grp[0], t); break;
      case 3: derived_digit_pieces<8>(hist, plan->nbins, q, s_grp[0], t); break;
      case 4: derived_digit_pieces<16>(hist, plan->nbins, q, s_grp[0], t); break;
      case 5: derived_digit_pieces<32>(hist, plan->nbins, q, s_grp[0], t); break;
      default: derived_digit_pieces<64>(hist, plan->nbins, q, s_grp[0], t); break;
    }
  }
  __syncthreads();
  if (t < 256) {
    c = 0;
#pragma unroll
    for (int i = 0; i < G; ++i) c += s_grp[i][d];
  }
  uint32_t total;
  const uint32_t ex = block_excl_scan<DIGIT_REDUCE_THREADS>(t < 256 ? c : 0u, s_scan, total);
  if (t < 256) {
    counts[p * 256 + d] = c;
    offsets[p * 256 + d] = ex;
  }
}

hipError_t launch_digit_reduce(const uint32_t* digit_partials, const uint32_t* hist, int nblocks, int ndig,
                               uint32_t* counts, uint32_t* offsets, hipStream_t s, const DevFeatures* plan,
                               const double* hpart, int nparts, DevFeatures* df) {
  if (plan && !hist) return hipErrorInvalidValue;  // derived digits read the reduced histogram
  if (hpart && !df) return hipErrorInvalidValue;
  const int nb = plan ? 8 : ndig;
  if (nb < 1) return hipErrorInvalidValue;
  k_digit_reduce<<<nb, DIGIT_REDUCE_THREADS, 0, s>>>(digit_partials, hist, nblocks, ndig, counts, offsets, plan,
                                                     hpart, nparts, df);
  return hipGetLastError();
}

}  // namespace ahs
