// Batched sort, large segments: features and the decision of Sec. III-A
// before sorting, then the kernel family the decision names.
//
//   min/max   one chunked pass over every large segment (SEG_CH keys per
//             workgroup), mapped keys, NaN count; per-segment atomics.
//   decide    one thread per large segment: NaN -> its bit-map order via the
//             sample sort; a forced strategy; COUNTING when the span is below
//             k_count; QUICK when it is below k_radix; otherwise the segment
//             joins the hist list, whose entropy decides RADIX or QUICK.
//   hist      one workgroup per unit of a hist-list segment (the whole
//             segment up to SEG_HU keys, else SEG_HU_MULTI keys at a time):
//             65,536 packed 16-bit LDS bins of (key - min) >> shift,
//             wraps repaired exactly from the atomics' return values (at most
//             SEG_HIST_EVENTS corrections per unit), then the FP64 entropy
//             and the decision; a segment of several units adds its units'
//             exact counts into a global histogram first.
//   radix     the COUNTING and RADIX segments: per-segment counts of the
//             8-bit digits of key - min, a pass plan per segment (digits that
//             are the same for every key skipped), then up to SEG_MAX_PASSES
//             stable onesweep passes whose tiles never cross a segment, with
//             one look-back chain per segment.  Segment s ping-pongs between
//             the output and the scratch buffer so that its last pass writes
//             the output.  A counting sort over at most 2^16 values is the
//             same stable scatter by the bin index: one or two digit passes.
#include "histcommon.hpp"
#include "onesweep.hpp"
#include "segmented.hpp"

namespace ahs {

namespace {

constexpr int SD_THREADS = 256;

__device__ __forceinline__ uint32_t seg_digits(uint64_t span) {
  const int d = (bitlen64(span) + 7) / 8;
  return d > 0 ? (uint32_t)d : 1u;
}

__device__ __forceinline__ void push_quick(const SegDispatchArgs& a, const SsSeg& g) {
  const uint32_t qi = atomicAdd(&a.qrec->nsegs_next, 1u);
  atomicAdd(&a.qrec->seg_keys_next, (unsigned long long)g.size);
  if (qi < a.qcap) {
    SsSeg q = g;
    q.first_tile = 0;
    a.qsegs[qi] = q;
  } else {
    atomicOr(&a.dctr->bad, 1u);
  }
}

__device__ __forceinline__ void push_radix(const SegDispatchArgs& a, const SsSeg& g, uint32_t li, uint64_t kmin,
                                           uint64_t span) {
  const uint32_t ri = atomicAdd(&a.dctr->radix.nsegs_next, 1u);
  if (ri >= a.list_cap) {
    atomicOr(&a.dctr->bad, 1u);
    return;
  }
  SsSeg r = g;
  r.first_tile = 0;
  a.rsegs[ri] = r;
  SegRadixInfo info = {};
  info.kmin = kmin;
  info.large = li;
  info.ndig = seg_digits(span);
  info.npass = 0;
  a.rinfo[ri] = info;
}

}  // namespace

// ------------------------------------------------------------------ min/max
template <int KK>
__global__ __launch_bounds__(SD_THREADS) void k_sd_minmax(SegDispatchArgs a) {
  using K = typename KeyTraits<KK>::K;
  constexpr int CPT = SEG_CH / SD_THREADS;
  uint32_t nch = a.chunks->ntiles_next;
  nch = nch < a.chunk_cap ? nch : a.chunk_cap;
  const uint32_t nl = a.chunks->nsegs_next;
  const int t = threadIdx.x;
  for (uint32_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const uint32_t li = ss_seg_of_tile(a.large, nl, c);
    const SsSeg g = a.large[li];
    const uint32_t c0 = (c - g.first_tile) * SEG_CH;
    const uint32_t cnt = g.size - c0 < SEG_CH ? g.size - c0 : SEG_CH;
    const K* __restrict__ keys = (const K*)a.kin + g.start + c0;
    K x[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const uint32_t j = (uint32_t)t + (uint32_t)q * SD_THREADS;
      x[q] = keys[j < cnt ? j : cnt - 1];
    }
    K mn = ~K(0), mx = K(0);
    uint32_t nan = 0;
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const uint32_t j = (uint32_t)t + (uint32_t)q * SD_THREADS;
      if (j < cnt) {
        if (KeyTraits<KK>::FLT && fnan(x[q])) {
          ++nan;
        } else {
          const K m = map_key<KK>(x[q]);
          mn = m < mn ? m : mn;
          mx = m > mx ? m : mx;
        }
      }
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    if constexpr (KeyTraits<KK>::FLT) nan = wave_sum(nan);
    if (lane_id() == 0) {
      atomicMin(&a.linfo[li].mn, (unsigned long long)mn);
      atomicMax(&a.linfo[li].mx, (unsigned long long)mx);
      if (nan) atomicAdd(&a.linfo[li].nan, nan);
    }
  }
}

// ------------------------------------------------------------------ decide
template <int KK>
__global__ __launch_bounds__(SD_THREADS) void k_sd_decide(SegDispatchArgs a) {
  const uint32_t count = a.ctr->bad ? 0u : a.ctr->nlarge;
  for (uint32_t i = blockIdx.x * SD_THREADS + threadIdx.x; i < count; i += gridDim.x * SD_THREADS) {
    const SsSeg g = a.large[i];
    const SegLarge L = a.linfo[i];
    const uint32_t s = a.large_ids[i];
    const uint64_t span = L.mx - L.mn;
    uint32_t chosen;
    int route;  // 0 quick, 1 radix, 2 hist
    if (L.nan) {
      chosen = SEG_STATUS_NAN;
      route = 0;
    } else if (a.requested) {
      chosen = a.requested;
      route = a.requested == 3u ? 0 : 1;
    } else if (g.size <= a.cfg.n_small) {
      chosen = 4u;  // INSERTION (a large segment under a large n_small): any stable sort realises it
      route = 0;
    } else if (span <= a.cfg.k_count - 1) {
      chosen = 1u;  // COUNTING
      route = 1;
    } else if (span < a.cfg.k_radix) {
      chosen = 3u;  // QUICK: k <= k_radix
      route = 0;
    } else {
      chosen = 0u;  // entropy decides
      route = 2;
    }
    if (route != 2 && a.chosen) a.chosen[s] = (uint8_t)chosen;
    if (route == 0) {
      push_quick(a, g);
    } else if (route == 1) {
      push_radix(a, g, i, L.mn, span);
    } else {
      const uint32_t hi = atomicAdd(&a.dctr->hist.nsegs_next, 1u);
      if (hi >= a.list_cap) {
        atomicOr(&a.dctr->bad, 1u);
        continue;
      }
      SsSeg h = g;
      h.first_tile = 0;
      a.hsegs[hi] = h;
      a.hlarge[hi] = i;
      uint32_t slot = 0xFFFFFFFFu;
      if (g.size > SEG_HU) {
        slot = atomicAdd(&a.dctr->nslot, 1u);
        if (slot >= a.slot_cap) {
          atomicOr(&a.dctr->bad, 1u);
          slot = 0xFFFFFFFFu;
        }
      }
      a.hslot_of[hi] = slot;
    }
  }
}

// Numbers the histogram units of the hist list (first unit of each
// segment, total units), one workgroup: a segment takes one unit up to
// SEG_HU keys, else units of SEG_HU_MULTI keys.
constexpr int SD_UNITS_THREADS = 1024;
__global__ __launch_bounds__(SD_UNITS_THREADS) void k_sd_hist_units(SegDispatchArgs a) {
  __shared__ uint32_t sm[SD_UNITS_THREADS / WAVE + 1];
  uint32_t nh = a.dctr->hist.nsegs_next;
  nh = nh < a.list_cap ? nh : a.list_cap;
  const uint32_t per = (nh + SD_UNITS_THREADS - 1) / SD_UNITS_THREADS;
  const uint32_t s0 = threadIdx.x * per;
  auto units = [&](uint32_t size) { return (size + seg_hist_unit_keys(size) - 1) / seg_hist_unit_keys(size); };
  uint32_t local = 0;
  for (uint32_t i = 0; i < per; ++i)
    if (s0 + i < nh) local += units(a.hsegs[s0 + i].size);
  uint32_t total;
  uint32_t run = block_excl_scan<SD_UNITS_THREADS>(local, sm, total);
  for (uint32_t i = 0; i < per; ++i) {
    if (s0 + i < nh) {
      a.hsegs[s0 + i].first_tile = run;
      run += units(a.hsegs[s0 + i].size);
    }
  }
  if (threadIdx.x == 0) a.dctr->hist.ntiles_next = total;
}

// Clears the global histograms of the multi-unit hist-list segments.
__global__ __launch_bounds__(SD_THREADS) void k_sd_clear_slots(SegDispatchArgs a) {
  uint32_t ns = a.dctr->nslot;
  ns = ns < a.slot_cap ? ns : a.slot_cap;
  const uint64_t words = (uint64_t)ns * 65536u;
  u32x4* p = reinterpret_cast<u32x4*>(a.hslots);
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (uint64_t i = (uint64_t)blockIdx.x * SD_THREADS + threadIdx.x; i < words / 4; i += (uint64_t)gridDim.x * SD_THREADS)
    p[i] = z;
}

// ------------------------------------------------------------------ hist
// Decision of a hist-list segment from its entropy; appends it to the list
// that sorts it.  Called by one thread.
__device__ __forceinline__ void sd_hist_decide(const SegDispatchArgs& a, uint32_t hidx, double H, uint32_t nbins) {
  const uint32_t li = a.hlarge[hidx];
  const SsSeg g = a.large[li];
  const SegLarge L = a.linfo[li];
  const uint64_t span = L.mx - L.mn;
  const uint8_t c = seg_fsm(g.size, span, nbins, H < 0.0 ? 0.0 : H, a.cfg);
  if (a.chosen) a.chosen[a.large_ids[li]] = c;
  if (c == 2) push_radix(a, g, li, L.mn, span); else push_quick(a, g);
}

template <int NT>
__device__ __forceinline__ double block_sum_f64(double v, double* smem) {
  v = wave_sum(v);
  if (lane_id() == 0) smem[threadIdx.x / WAVE] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / WAVE; ++i) s += smem[i];
  return s;  // valid in thread 0
}

template <int KK>
__global__ __launch_bounds__(SEG_HIST_THREADS) void k_sd_hist(SegDispatchArgs a) {
  using K = typename KeyTraits<KK>::K;
  constexpr int V = 16 / sizeof(K);
  constexpr int NT = SEG_HIST_THREADS;
  __shared__ uint32_t h[HIST_LARGE_WORDS];   // bin 2w in the low half of word w, 2w+1 in the high half
  __shared__ uint32_t s_bm[65536 / 32];      // bins with corrections
  __shared__ uint32_t s_evb[SEG_HIST_EVENTS], s_evd[SEG_HIST_EVENTS];
  __shared__ uint32_t s_nev;
  __shared__ double s_red[NT / WAVE];
  static_assert(sizeof(h) + sizeof(s_bm) + 2 * sizeof(s_evb) + sizeof(s_red) + 16 <= 160 * 1024, "LDS");
  uint32_t nu = a.dctr->hist.ntiles_next;
  nu = nu < a.unit_cap ? nu : a.unit_cap;
  uint32_t nh = a.dctr->hist.nsegs_next;
  nh = nh < a.list_cap ? nh : a.list_cap;
  const int t = threadIdx.x;
  for (uint32_t u = blockIdx.x; u < nu; u += gridDim.x) {
    __syncthreads();  // the previous unit's LDS contents are consumed
    for (int i = t; i < HIST_LARGE_WORDS; i += NT) h[i] = 0u;
    for (int i = t; i < 65536 / 32; i += NT) s_bm[i] = 0u;
    if (t == 0) s_nev = 0u;
    const uint32_t hidx = ss_seg_of_tile(a.hsegs, nh, u);
    const SsSeg hg = a.hsegs[hidx];
    const uint32_t li = a.hlarge[hidx];
    const SegLarge L = a.linfo[li];
    const K kmin = (K)L.mn;
    uint32_t shift, nbins;
    shift_nbins(L.mx - L.mn, shift, nbins);
    const uint32_t ukeys = seg_hist_unit_keys(hg.size);
    const uint64_t u0 = (uint64_t)(u - hg.first_tile) * ukeys;
    const uint32_t cnt = (uint32_t)((uint64_t)hg.size - u0 < ukeys ? (uint64_t)hg.size - u0 : ukeys);
    const bool multi = hg.size > SEG_HU;
    __syncthreads();

    auto record = [&](uint32_t bin, uint32_t delta) {
      const uint32_t e = atomicAdd(&s_nev, 1u);
      if (e < (uint32_t)SEG_HIST_EVENTS) {
        s_evb[e] = bin;
        s_evd[e] = delta;
      }
      atomicOr(&s_bm[bin >> 5], 1u << (bin & 31u));
    };
    // additive corrections modulo 2^32 after c was added to `bin`, whose
    // word held `old`: a low-half wrap moves 65,536 into the bin and takes
    // back the carry that leaked into the high half (which itself wraps when
    // the high half was full); a high-half wrap moves 65,536 into the bin
    auto fix_packed = [&](uint32_t bin, uint32_t old, uint32_t c) {
      if (bin & 1u) {
        if ((old >> 16) + c > 0xFFFFu) record(bin, 65536u);
      } else if ((old & 0xFFFFu) + c > 0xFFFFu) {
        record(bin, 65536u);
        record(bin + 1, (old >> 16) == 0xFFFFu ? 65535u : 0xFFFFFFFFu);
      }
    };
    auto packed_add = [&](uint32_t bin, uint32_t c) { return atomicAdd(&h[bin >> 1], (bin & 1u) ? (c << 16) : c); };

    const K* __restrict__ keys = (const K*)a.kin + hg.start + u0;
    for_each_group<K, 4>(keys, cnt, (uint64_t)t, (uint64_t)NT, [&](const K (&kb)[V], int m) {
      uint32_t bins[V];
      bool pend[V];
#pragma unroll
      for (int i = 0; i < V; ++i) {
        bins[i] = (uint32_t)((map_key<KK>(kb[i]) - kmin) >> shift);
        pend[i] = i < m;
      }
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
    });
    __syncthreads();
    const uint32_t nev = s_nev < (uint32_t)SEG_HIST_EVENTS ? s_nev : (uint32_t)SEG_HIST_EVENTS;
    if (t == 0 && s_nev > (uint32_t)SEG_HIST_EVENTS) atomicOr(&a.dctr->bad, 1u);  // cannot happen: cnt <= SEG_HU
    auto count_of = [&](uint32_t b) {
      const uint32_t w = h[b >> 1];
      uint32_t c = (b & 1u) ? (w >> 16) : (w & 0xFFFFu);
      if (s_bm[b >> 5] & (1u << (b & 31u)))
        for (uint32_t e = 0; e < nev; ++e)
          if (s_evb[e] == b) c += s_evd[e];
      return c;
    };
    if (!multi) {
      const double inv_n = 1.0 / (double)hg.size;
      double acc = 0.0;
      for (uint32_t b = (uint32_t)t; b < nbins; b += NT) {
        const uint32_t c = count_of(b);
        if (c) {
          const double p = (double)c * inv_n;
          acc -= p * log2(p);
        }
      }
      const double H = block_sum_f64<NT>(acc, s_red);
      if (t == 0) sd_hist_decide(a, hidx, H, nbins);
    } else {
      const uint32_t slot = a.hslot_of[hidx];
      if (slot != 0xFFFFFFFFu) {
        uint32_t* __restrict__ gh = a.hslots + (size_t)slot * 65536u;
        for (uint32_t b = (uint32_t)t; b < nbins; b += NT) {
          const uint32_t c = count_of(b);
          if (c) atomicAdd(&gh[b], c);
        }
      }
    }
  }
}

// Entropy and decision of the multi-unit hist-list segments, from their
// global histograms; one workgroup per segment.
__global__ __launch_bounds__(SD_THREADS) void k_sd_hist_final(SegDispatchArgs a) {
  __shared__ double s_red[SD_THREADS / WAVE];
  uint32_t nh = a.dctr->hist.nsegs_next;
  nh = nh < a.list_cap ? nh : a.list_cap;
  const int t = threadIdx.x;
  for (uint32_t hidx = blockIdx.x; hidx < nh; hidx += gridDim.x) {
    const SsSeg hg = a.hsegs[hidx];
    if (hg.size <= SEG_HU) continue;  // decided by its single unit
    const uint32_t slot = a.hslot_of[hidx];
    const SegLarge L = a.linfo[a.hlarge[hidx]];
    uint32_t shift, nbins;
    shift_nbins(L.mx - L.mn, shift, nbins);
    double acc = 0.0;
    if (slot != 0xFFFFFFFFu) {
      const uint32_t* __restrict__ gh = a.hslots + (size_t)slot * 65536u;
      const double inv_n = 1.0 / (double)hg.size;
      for (uint32_t b = (uint32_t)t; b < nbins; b += SD_THREADS) {
        const uint32_t c = gh[b];
        if (c) {
          const double p = (double)c * inv_n;
          acc -= p * log2(p);
        }
      }
    }
    __syncthreads();
    const double H = block_sum_f64<SD_THREADS>(acc, s_red);
    if (t == 0) sd_hist_decide(a, hidx, H, nbins);
  }
}

// ------------------------------------------------------------------ radix: digit counts and plan
__global__ __launch_bounds__(SD_THREADS) void k_sd_rclear(SegDispatchArgs a) {
  uint32_t nr = a.dctr->radix.nsegs_next;
  nr = nr < a.list_cap ? nr : a.list_cap;
  const uint64_t words = (uint64_t)nr * 8u * 256u;
  u32x4* p = reinterpret_cast<u32x4*>(a.rdig);
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (uint64_t i = (uint64_t)blockIdx.x * SD_THREADS + threadIdx.x; i < words / 4; i += (uint64_t)gridDim.x * SD_THREADS)
    p[i] = z;
}

template <int KK>
__global__ __launch_bounds__(SEG_RD_THREADS) void k_sd_rdigits(SegDispatchArgs a, uint32_t tile_keys) {
  using K = typename KeyTraits<KK>::K;
  constexpr int V = 16 / sizeof(K);
  constexpr int DMAX = sizeof(K);
  __shared__ uint32_t s_cnt[DMAX * 256];
  uint32_t ntiles = a.dctr->radix.ntiles_next;
  ntiles = ntiles < a.tile_cap ? ntiles : a.tile_cap;
  uint32_t nr = a.dctr->radix.nsegs_next;
  nr = nr < a.list_cap ? nr : a.list_cap;
  const int t = threadIdx.x;
  for (uint32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    __syncthreads();
    for (int i = t; i < DMAX * 256; i += SEG_RD_THREADS) s_cnt[i] = 0u;
    const uint32_t r = ss_seg_of_tile(a.rsegs, nr, tile);
    const SsSeg g = a.rsegs[r];
    const SegRadixInfo info = a.rinfo[r];
    const int ndig = (int)(info.ndig < (uint32_t)DMAX ? info.ndig : (uint32_t)DMAX);
    const K kmin = (K)info.kmin;
    const uint64_t off = (uint64_t)(tile - g.first_tile) * tile_keys;
    const uint32_t cnt = (uint32_t)((uint64_t)g.size - off < tile_keys ? (uint64_t)g.size - off : tile_keys);
    __syncthreads();
    const K* __restrict__ keys = (const K*)a.kin + g.start + off;
    for_each_group<K, 2>(keys, cnt, (uint64_t)t, (uint64_t)SEG_RD_THREADS, [&](const K (&kb)[V], int m) {
      K o[V];
#pragma unroll
      for (int i = 0; i < V; ++i) o[i] = map_key<KK>(kb[i]) - kmin;
      for (int p = 0; p < ndig; ++p) {
        uint32_t dg[V];
#pragma unroll
        for (int i = 0; i < V; ++i) dg[i] = (uint32_t)((o[i] >> (8 * p)) & 255u);
        lds_count_group<V>(s_cnt + p * 256, dg, m);
      }
    });
    __syncthreads();
    uint32_t* __restrict__ out = a.rdig + (size_t)r * 8u * 256u;
    for (int i = t; i < ndig * 256; i += SEG_RD_THREADS)
      if (s_cnt[i]) atomicAdd(&out[i], s_cnt[i]);
  }
}

// Per radix segment: exclusive digit offsets (in place of the counts), the
// digits that move keys, and the pass list.  With keys or payload sorted in
// place an odd pass count gets its first pass repeated (sorting by the same
// digit twice is the identity on the second pass) so that the first pass
// writes the scratch buffer and the last one the output.
__global__ __launch_bounds__(256) void k_sd_rplan(SegDispatchArgs a) {
  __shared__ uint32_t s_scan[256 / WAVE + 1];
  __shared__ uint32_t s_triv[8];
  uint32_t nr = a.dctr->radix.nsegs_next;
  nr = nr < a.list_cap ? nr : a.list_cap;
  const int t = threadIdx.x;
  for (uint32_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const SsSeg g = a.rsegs[r];
    const uint32_t ndig = a.rinfo[r].ndig;
    uint32_t* __restrict__ dig = a.rdig + (size_t)r * 8u * 256u;
    __syncthreads();
    if (t < 8) s_triv[t] = 0u;
    __syncthreads();
    for (uint32_t p = 0; p < ndig; ++p) {
      const uint32_t c = dig[p * 256 + t];
      if (c == g.size) s_triv[p] = 1u;
      uint32_t total;
      const uint32_t ex = block_excl_scan<256>(c, s_scan, total);
      dig[p * 256 + t] = ex;
    }
    __syncthreads();
    if (t == 0) {
      SegRadixInfo info = a.rinfo[r];
      uint32_t np = 0;
      uint8_t ps[SEG_MAX_PASSES];
      for (uint32_t p = 0; p < ndig; ++p)
        if (!s_triv[p]) ps[np++] = (uint8_t)p;
      if (np == 0) ps[np++] = 0;  // every digit constant: one pass is a stable copy
      uint32_t k = 0;
      if (a.in_place && (np & 1u)) info.pass[k++] = ps[0];
      for (uint32_t i = 0; i < np; ++i) info.pass[k++] = ps[i];
      info.npass = k;
      a.rinfo[r] = info;
      atomicMax(&a.dctr->max_npass, k);
    }
  }
}

// ------------------------------------------------------------------ radix: one pass
template <int KK, bool PAY, int IPT, typename ST>
__global__ __launch_bounds__(SEG_RD_THREADS, 4) void k_sd_rpass(SegDispatchArgs a, int q) {
  using K = typename KeyTraits<KK>::K;
  constexpr int NT = SEG_RD_THREADS;
  constexpr int NW = NT / WAVE;
  constexpr int TILE = NT * IPT;
  constexpr size_t SLOT_BYTES = sizeof(RankLds<256>) * NW;
  constexpr size_t KEY_BYTES = sizeof(K) * TILE;
  static_assert(sizeof(uint32_t) * NW * 256 <= SLOT_BYTES, "position table fits over the slots");
  __shared__ __align__(16) unsigned char s_raw[SLOT_BYTES > KEY_BYTES ? SLOT_BYTES : KEY_BYTES];
  RankLds<256>* s_rank = reinterpret_cast<RankLds<256>*>(s_raw);
  uint32_t(*s_pos)[256] = reinterpret_cast<uint32_t(*)[256]>(s_raw);
  K* s_keys = reinterpret_cast<K*>(s_raw);
  __shared__ uint32_t s_dadj[256];
  __shared__ uint32_t s_vals[PAY ? TILE : 1];
  __shared__ uint32_t s_scan[NW + 1];
  __shared__ uint32_t s_tile;

  if ((uint32_t)q >= a.dctr->max_npass) return;  // no segment has this many passes
  uint32_t ntiles = a.dctr->radix.ntiles_next;
  ntiles = ntiles < a.tile_cap ? ntiles : a.tile_cap;
  uint32_t nr = a.dctr->radix.nsegs_next;
  nr = nr < a.list_cap ? nr : a.list_cap;
  const int t = threadIdx.x, w = t / WAVE;
  for (;;) {
    __syncthreads();  // the previous tile's LDS contents are consumed
    rank_clear<256, NT>(s_rank, NW);
    if (t == 0) s_tile = add_agent(&a.dctr->tile_ctr[1 + q], 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) break;
    const uint32_t rs = ss_seg_of_tile(a.rsegs, nr, tile);
    const SsSeg sg = a.rsegs[rs];
    const SegRadixInfo& info = a.rinfo[rs];
    const uint32_t npass = info.npass;
    if ((uint32_t)q >= npass) continue;  // this segment is done (the same for the whole workgroup)
    const uint32_t shift = 8u * info.pass[q];
    const K kmin = (K)info.kmin;
    const bool to_out = ((npass - 1u - (uint32_t)q) & 1u) == 0u;
    const bool from_out = ((npass - (uint32_t)q) & 1u) == 0u;  // where pass q - 1 wrote
    const uint64_t off = (uint64_t)(tile - sg.first_tile) * TILE;
    // tile-relative source and segment-relative destination: 32-bit offsets from uniform bases
    const K* __restrict__ src =
        (const K*)(q == 0 ? a.kin : (from_out ? (const void*)a.kout : (const void*)a.ktmp)) + sg.start + off;
    K* __restrict__ dst = (K*)(to_out ? a.kout : a.ktmp) + sg.start;
    const uint32_t* __restrict__ vsrc = PAY ? (q == 0 ? a.vin : (from_out ? a.vout : a.vtmp)) + sg.start + off : nullptr;
    uint32_t* __restrict__ vdst = PAY ? (to_out ? a.vout : a.vtmp) + sg.start : nullptr;
    const bool map_in = key_mapped<KK> && q == 0;
    const bool unmap_out = key_mapped<KK> && (uint32_t)q == npass - 1u;
    const uint64_t rem = (uint64_t)sg.size - off;
    const uint32_t valid = rem < (uint64_t)TILE ? (uint32_t)rem : (uint32_t)TILE;
    const uint32_t dbase = (uint32_t)(t < 256 ? a.rdig[(size_t)rs * 8u * 256u + info.pass[q] * 256u + t] : 0u);
    auto digit = [&](K x) { return (uint32_t)(((x - kmin) >> shift) & 255u); };

    // thread and lane ids made opaque per tile: otherwise the compiler hoists
    // the IPT per-item offsets out of the tile loop and holds them in VGPRs
    uint32_t tv = (uint32_t)t;
    asm volatile("" : "+v"(tv));
    const uint32_t lane = tv & (WAVE - 1);
    K k[IPT];
    uint32_t v[IPT];
    const uint32_t wbase = (uint32_t)w * WAVE * IPT;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t idx = wbase + (uint32_t)i * WAVE + lane;
      const uint32_t ci = idx < valid ? idx : valid - 1;
      k[i] = src[ci];
      if constexpr (PAY) v[i] = vsrc[ci];
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t idx = wbase + (uint32_t)i * WAVE + lane;
      K x = k[i];
      if constexpr (key_mapped<KK>) x = map_in ? map_key<KK>(x) : x;
      // padding: a key of digit 255, ranked after every real key of the tile
      if (idx >= valid) x = kmin + (K)((K)255 << shift);
      k[i] = x;
    }
    uint32_t r[IPT];
    {
      uint32_t d[IPT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) d[i] = digit(k[i]);
      rank_wave_items<IPT>(d, r, s_rank[w]);
    }
    __syncthreads();

    uint32_t cnt = 0, wpre[NW];
    if (t < 256) {
#pragma unroll
      for (int u = 0; u < NW; ++u) {
        wpre[u] = cnt;
        cnt += s_rank[u].count[t];
      }
      if (t == 255) cnt -= (uint32_t)TILE - valid;
    }
    uint32_t total;
    const uint32_t tstart = block_excl_scan<NT>(t < 256 ? cnt : 0u, s_scan, total);
    if (t < 256) {
#pragma unroll
      for (int u = 0; u < NW; ++u) s_pos[u][t] = wpre[u] + tstart;
      const uint64_t excl = lookback<256, ST>((ST*)a.status, tile, sg.first_tile, (uint32_t)t, cnt);
      s_dadj[t] = dbase + (uint32_t)excl - tstart;  // modulo 2^32; + j lands in [0, size)
    }
    __syncthreads();
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
    __syncthreads();

    auto put = [&](uint32_t j, K x, uint32_t rel) {
      if (rel >= sg.size) return;  // padding
      if constexpr (key_mapped<KK>) x = unmap_out ? unmap_key<KK>(x) : x;
      dst[rel] = x;
      if constexpr (PAY) vdst[rel] = s_vals[j];
    };
    if (valid == (uint32_t)TILE) {
      K x[IPT];
      uint32_t o[IPT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) x[i] = s_keys[tv + i * NT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) o[i] = s_dadj[digit(x[i])] + (tv + (uint32_t)(i * NT));
#pragma unroll
      for (int i = 0; i < IPT; ++i) put(tv + (uint32_t)(i * NT), x[i], o[i]);
    } else {
      for (uint32_t j = t; j < valid; j += NT) {
        const K x = s_keys[j];
        put(j, x, s_dadj[digit(x)] + j);
      }
    }
  }
}

// Clears the look-back words of the radix tiles before a pass.
__global__ __launch_bounds__(SD_THREADS) void k_sd_zero_status(SegDispatchArgs a, uint32_t words_per_tile, int q) {
  if ((uint32_t)q >= a.dctr->max_npass) return;
  uint32_t ntiles = a.dctr->radix.ntiles_next;
  ntiles = ntiles < a.tile_cap ? ntiles : a.tile_cap;
  const uint64_t nvec = (uint64_t)ntiles * words_per_tile / 4;
  u32x4* p = static_cast<u32x4*>(a.status);
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (uint64_t i = (uint64_t)blockIdx.x * SD_THREADS + threadIdx.x; i < nvec; i += (uint64_t)gridDim.x * SD_THREADS)
    p[i] = z;
}

// ------------------------------------------------------------------ launchers
namespace {

template <typename Kern>
uint32_t resident_blocks(Kern k, int threads, uint32_t cu_count) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  return (uint32_t)per_cu * (cu_count ? cu_count : 256u);
}

template <int KK>
hipError_t dispatch_kk(const SegDispatchArgs& a, uint32_t cu, hipStream_t s) {
  const uint32_t grid = 4 * (cu ? cu : 256u);
  k_sd_minmax<KK><<<grid * 4, SD_THREADS, 0, s>>>(a);
  k_sd_decide<KK><<<grid, SD_THREADS, 0, s>>>(a);
  k_sd_hist_units<<<1, SD_UNITS_THREADS, 0, s>>>(a);
  k_sd_clear_slots<<<grid, SD_THREADS, 0, s>>>(a);
  k_sd_hist<KK><<<resident_blocks(k_sd_hist<KK>, SEG_HIST_THREADS, cu), SEG_HIST_THREADS, 0, s>>>(a);
  k_sd_hist_final<<<grid, SD_THREADS, 0, s>>>(a);
  return hipGetLastError();
}

template <int KK>
hipError_t radix_prepare_kk(const SegDispatchArgs& a, uint32_t tile_keys, uint32_t cu, hipStream_t s) {
  const uint32_t grid = 4 * (cu ? cu : 256u);
  hipError_t e = launch_ss_tiles(a.rsegs, &a.dctr->radix, tile_keys, a.list_cap, s);
  if (e != hipSuccess) return e;
  k_sd_rclear<<<grid, SD_THREADS, 0, s>>>(a);
  k_sd_rdigits<KK><<<resident_blocks(k_sd_rdigits<KK>, SEG_RD_THREADS, cu), SEG_RD_THREADS, 0, s>>>(a, tile_keys);
  k_sd_rplan<<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

// Tile shapes of the radix passes: two per key size and payload flag.
constexpr int RD_IPT[2][2][2] = {{{16, 24}, {12, 18}}, {{12, 18}, {8, 12}}};  // [8-byte keys][payload][variant]

template <int KK, bool PAY, int IPT, typename ST>
hipError_t rpass_launch(const SegDispatchArgs& a, int q, uint32_t cu, hipStream_t s) {
  static_assert(IPT >= 8, "radix tiles of at least 4,096 keys: their look-back words fit the sample sort's");
  const uint32_t words = 256 * (uint32_t)sizeof(ST) / 4;
  k_sd_zero_status<<<4 * (cu ? cu : 256u), SD_THREADS, 0, s>>>(a, words, q);
  static uint32_t per_cu = 0;  // resident workgroups per CU, looked up once
  if (!per_cu) per_cu = resident_blocks(k_sd_rpass<KK, PAY, IPT, ST>, SEG_RD_THREADS, 1u);
  k_sd_rpass<KK, PAY, IPT, ST><<<per_cu * (cu ? cu : 256u), SEG_RD_THREADS, 0, s>>>(a, q);
  return hipGetLastError();
}

template <int KK, bool PAY>
hipError_t rpass_kk(int variant, const SegDispatchArgs& a, int q, uint64_t max_seg, uint32_t cu, hipStream_t s) {
  constexpr int KB = sizeof(typename KeyTraits<KK>::K) == 8 ? 1 : 0;
  const bool wide = max_seg >= STATUS32_MAX_N;
  if (variant == 0) {
    constexpr int IPT = RD_IPT[KB][PAY ? 1 : 0][0];
    return wide ? rpass_launch<KK, PAY, IPT, uint64_t>(a, q, cu, s) : rpass_launch<KK, PAY, IPT, uint32_t>(a, q, cu, s);
  }
  constexpr int IPT = RD_IPT[KB][PAY ? 1 : 0][1];
  return wide ? rpass_launch<KK, PAY, IPT, uint64_t>(a, q, cu, s) : rpass_launch<KK, PAY, IPT, uint32_t>(a, q, cu, s);
}

}  // namespace

uint32_t seg_radix_tile(int key_bytes, int with_vals, int ipt_variant) {
  return (uint32_t)SEG_RD_THREADS * (uint32_t)RD_IPT[key_bytes == 8 ? 1 : 0][with_vals ? 1 : 0][ipt_variant ? 1 : 0];
}

hipError_t launch_seg_dispatch(int kk, const SegDispatchArgs& a, uint32_t cu_count, hipStream_t s) {
  switch (kk) {
    case KK_U32: return dispatch_kk<KK_U32>(a, cu_count, s);
    case KK_U64: return dispatch_kk<KK_U64>(a, cu_count, s);
    case KK_F32: return dispatch_kk<KK_F32>(a, cu_count, s);
    case KK_F64: return dispatch_kk<KK_F64>(a, cu_count, s);
    case KK_I32: return dispatch_kk<KK_I32>(a, cu_count, s);
    case KK_I64: return dispatch_kk<KK_I64>(a, cu_count, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_seg_radix_prepare(int kk, const SegDispatchArgs& a, uint32_t tile_keys, uint32_t cu_count,
                                    hipStream_t s) {
  switch (kk) {
    case KK_U32: return radix_prepare_kk<KK_U32>(a, tile_keys, cu_count, s);
    case KK_U64: return radix_prepare_kk<KK_U64>(a, tile_keys, cu_count, s);
    case KK_F32: return radix_prepare_kk<KK_F32>(a, tile_keys, cu_count, s);
    case KK_F64: return radix_prepare_kk<KK_F64>(a, tile_keys, cu_count, s);
    case KK_I32: return radix_prepare_kk<KK_I32>(a, tile_keys, cu_count, s);
    case KK_I64: return radix_prepare_kk<KK_I64>(a, tile_keys, cu_count, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_seg_radix_pass(int kk, int with_vals, int ipt_variant, const SegDispatchArgs& a, int q,
                                 uint64_t max_seg, uint32_t cu_count, hipStream_t s) {
  if (q < 0 || q >= SEG_MAX_PASSES) return hipErrorInvalidValue;
  switch (kk * 2 + (with_vals ? 1 : 0)) {
    case KK_U32 * 2: return rpass_kk<KK_U32, false>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_U32 * 2 + 1: return rpass_kk<KK_U32, true>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_U64 * 2: return rpass_kk<KK_U64, false>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_U64 * 2 + 1: return rpass_kk<KK_U64, true>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_F32 * 2: return rpass_kk<KK_F32, false>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_F32 * 2 + 1: return rpass_kk<KK_F32, true>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_F64 * 2: return rpass_kk<KK_F64, false>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_F64 * 2 + 1: return rpass_kk<KK_F64, true>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_I32 * 2: return rpass_kk<KK_I32, false>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_I32 * 2 + 1: return rpass_kk<KK_I32, true>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_I64 * 2: return rpass_kk<KK_I64, false>(ipt_variant, a, q, max_seg, cu_count, s);
    case KK_I64 * 2 + 1: return rpass_kk<KK_I64, true>(ipt_variant, a, q, max_seg, cu_count, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ahs
