// General path on gfx950: a stable GPU sample sort, the multi-pivot form of
// the paper's quicksort (Sec. III-G.1, Listing 4).  Where quicksort splits a
// range around one median-of-three pivot into <, == and >, each level here
// splits every active segment around 255 pivots (splitters) drawn from a
// sample, into 255 open intervals and 255 "equal to splitter" buckets, with
// a stable scatter; equal-key buckets are final, buckets of at most
// SS_CAP keys are finished by an in-LDS stable block sort, larger ones form
// the next level's segments.
//
// Bucket id of key x against sorted splitters s_0 <= ... <= s_254:
//   r = #{i : s_i < x};  id = 2r + (r < 255 && x == s_r)
// so ids ascend with the key and duplicate splitters only leave buckets
// empty.
#include <type_traits>

#include "blocksort.hpp"
#include "onesweep.hpp"
#include "samplesort.hpp"

namespace ahs {

// Bucket classification.  A key's bucket id is 2r + (x equals the r-th
// splitter), r = #{s_i < x} over the sorted splitters s_0 <= ... <= s_254.
//
// Cell table (most segments).  The range [s_0, s_254] is cut into C cells
// (1,024 for 32-bit keys, 512 for 64-bit) of 2^shift values from s_0 (the
// smallest shift that covers it).  cnt[c] = #{i : cell(s_i) < c}, c = 0..C,
// is a non-decreasing step
// function, so the splitters inside cell c are exactly those of index
// [cnt[c], cnt[c + 1]); a key x in cell c has r = cnt[c] + #{i in [cnt[c],
// cnt[c + 1]) : s_i < x}, a search over the few splitters of its own cell
// (none or one for most keys) in place of eight steps over all 255.  A key
// at or below s_0 has r = 0, a key past the last cell r = 255.
//
// Search tree (segments whose splitters crowd into cells: more than
// SS_CELL_MAX in one, as skewed or duplicate-heavy keys give).  The 255
// splitters as an implicit perfect search tree: node k (1..255) has children
// 2k and 2k + 1, in-order traversal gives ascending order, and node k at
// depth d holds the splitter of sorted index (2 (k - 2^d) + 1) 2^(7-d) - 1.
// A search reads one node per level, and the nodes of a level are
// consecutive words, so the 64 lanes of a wave read distinct LDS banks (or
// broadcast) where a binary search of the sorted array would hit one bank
// from many lanes.
//
// The sample kernel writes both layouts, the cell table and the choice into
// the segment's splitter record (ss_spl_rec_bytes); the count and scatter
// kernels load the layout the record names.
constexpr uint32_t SS_CELL_MAX = 16;
constexpr uint32_t SS_TREE = 0x80000000u;  // layout flag in the record's shift word
constexpr uint32_t SS_EQOUT = 0x40000000u;  // the plan marked buckets that go straight to the output
constexpr uint32_t SS_WORD_FLAGS = SS_TREE | SS_EQOUT;

__host__ __device__ __forceinline__ uint32_t ss_tree_sorted_index(uint32_t k) {
  const uint32_t d = 31u - (uint32_t)__builtin_clz(k);
  return ((2u * (k - (1u << d)) + 1u) << (7u - d)) - 1u;
}

template <typename K>
struct SsCells {
  K spl[256];                      // sorted splitters (0..254), or the tree (nodes 1..255)
  uint32_t cntw[ss_cell_words((int)sizeof(K))];  // cell table: cnt[c] as bytes
  __device__ const uint8_t* cnt() const { return reinterpret_cast<const uint8_t*>(cntw); }
};

// Loads the layout a segment's record names into LDS (every thread takes
// part; the caller places a barrier before the first use) and returns the
// record's word (shift | SS_TREE).
template <typename K, int NT>
__device__ __forceinline__ uint32_t ss_cells_load(SsCells<K>& c, const void* spl, uint32_t sidx) {
  const uint32_t su = __builtin_amdgcn_readfirstlane(sidx);  // a scalar load of the word
  const unsigned char* rec = static_cast<const unsigned char*>(spl) + (size_t)su * ss_spl_rec_bytes((int)sizeof(K));
  const uint32_t* rw = reinterpret_cast<const uint32_t*>(rec + sizeof(K) * 512);
  const uint32_t word = rw[ss_cell_words((int)sizeof(K))];
  if (word & SS_TREE) {
    const K* rt = reinterpret_cast<const K*>(rec) + 256;
    for (int k = (int)threadIdx.x; k < 256; k += NT) c.spl[k] = rt[k];
  } else {
    const K* rs = reinterpret_cast<const K*>(rec);
    for (int k = (int)threadIdx.x; k < SS_P; k += NT) c.spl[k] = rs[k];
    for (int k = (int)threadIdx.x; k < (int)ss_cell_words((int)sizeof(K)); k += NT) c.cntw[k] = rw[k];
  }
  return word;
}

// The record's output mask: bit b marks bucket b (valid when the word holds
// SS_EQOUT).
template <typename K>
__device__ __forceinline__ const uint32_t* ss_eq_mask(const void* spl, uint32_t sidx) {
  const unsigned char* rec = static_cast<const unsigned char*>(spl) + (size_t)sidx * ss_spl_rec_bytes((int)sizeof(K));
  return reinterpret_cast<const uint32_t*>(rec + ss_eq_mask_offset((int)sizeof(K)));
}

// Bucket id of x in the layout TREE names (the caller branches once per
// tile on the record's word).  base = s_0 and shift: the cell layout's.
template <bool TREE, typename K>
__device__ __forceinline__ uint32_t ss_classify(K x, const SsCells<K>& c, K base, uint32_t shift) {
  if constexpr (TREE) {
    const K* tree = c.spl;
    uint32_t k = 1;
#pragma unroll
    for (int l = 0; l < 8; ++l) k = 2u * k + (tree[k] < x ? 1u : 0u);
    const uint32_t r = k - 256u;
    // node of sorted index r: r + 1 = (2m + 1) 2^z puts it at depth 7 - z
    const uint32_t z = (uint32_t)__builtin_ctz(r + 1u);
    const uint32_t node = (1u << (7u - z)) + ((r + 1u) >> (z + 1u));
    const uint32_t eq = (r < (uint32_t)SS_P && tree[node] == x) ? 1u : 0u;
    return 2u * r + eq;
  }
  uint32_t r;
  if (x <= base) {
    r = 0;
  } else {
    const K cell = (x - base) >> shift;
    if (cell >= (K)(1u << ss_cells_log2((int)sizeof(K)))) {
      r = (uint32_t)SS_P;
    } else {
      const uint8_t* cnt = c.cnt();
      uint32_t lo = cnt[(uint32_t)cell], hi = cnt[(uint32_t)cell + 1u];
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (c.spl[mid] < x) lo = mid + 1u; else hi = mid;
      }
      r = lo;
    }
  }
  const uint32_t eq = (r < (uint32_t)SS_P && c.spl[r] == x) ? 1u : 0u;
  return 2u * r + eq;
}

__device__ __forceinline__ uint64_t ss_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}


// ------------------------------------------------------------------ init
// Level 0: one segment (or, for n <= SS_CAP, one block-sort item) covering
// the whole input.
// Clears the per-level counter records and tile counters and, with segs
// set, makes the whole input segment 0 and item 0 (one launch for all the
// set-up a sort needs).
__global__ void k_ss_init(SsSeg* segs, SsItem* items, uint64_t n, uint32_t* ctr_words, uint32_t nctr,
                          uint32_t* tilectr, uint32_t ntile) {
  for (uint32_t i = threadIdx.x; i < nctr; i += blockDim.x) ctr_words[i] = 0u;
  for (uint32_t i = threadIdx.x; i < ntile; i += blockDim.x) tilectr[i] = 0u;
  if (segs && threadIdx.x == 0 && blockIdx.x == 0) {
    segs[0].start = 0;
    segs[0].size = (uint32_t)n;
    segs[0].first_tile = 0;
    items[0].start = 0;
    items[0].size = (uint32_t)n;
    items[0].flags = SS_BUF_IN << 8;
  }
}

// ------------------------------------------------------------------ sample + splitters
// One block per segment (grid stride).  A segment of `size` keys gets
// q = size / SS_TARGET splitters (clamped to [1, SS_P]): about q + 1 ranges
// of SS_TARGET keys, so a medium segment splits into a few block-sort
// buckets instead of 511 tiny ones.  The sample holds about 32 keys per
// range, ns = 32 (q + 1) rounded up to a power of two in [512, SS_SAMPLES],
// drawn at pseudo-random positions and sorted by the in-LDS block sort.
// Splitter i (ascending) is sample (floor(i q / 255) + 1) ns / (q + 1):
// q distinct positions, each repeated; repeated splitters only leave
// buckets empty.  With q = 255, splitter i is sample (i + 1) ns / 256.
// Splitters are stored in both layouts of the bucket classification, with
// the cell table and the choice between them.  Also clears the bucket
// counts.
__host__ __device__ __forceinline__ uint32_t ss_splitters(uint32_t size) {
  const uint32_t q = size / (uint32_t)SS_TARGET;
  return q < 1u ? 1u : (q > (uint32_t)SS_P ? (uint32_t)SS_P : q);
}
__host__ __device__ __forceinline__ uint32_t ss_sample_size(uint32_t q) {
  uint32_t ns = (uint32_t)SS_THREADS;
  while (ns < 32u * (q + 1u) && ns < (uint32_t)SS_SAMPLES) ns <<= 1;
  return ns;
}

template <int KK>
__global__ __launch_bounds__(SS_THREADS) void k_ss_sample(const typename KeyTraits<KK>::K* __restrict__ src,
                                                          int map_in, const SsSeg* __restrict__ segs, SsLevelIn lv,
                                                          void* __restrict__ spl_rec,
                                                          uint32_t* __restrict__ counts, uint64_t seed) {
  using K = typename KeyTraits<KK>::K;
  using Smem = BlockSortSmem<K, false, SS_SAMPLES, SS_THREADS>;
  constexpr int IPT = SS_SAMPLES / SS_THREADS;
  __shared__ Smem sm;
  __shared__ uint32_t s_occ[SS_THREADS / WAVE];
  const uint32_t t = threadIdx.x;
  const uint32_t nsegs = lv.segs_n();
  for (uint32_t sidx = blockIdx.x; sidx < nsegs; sidx += gridDim.x) {
    __syncthreads();  // the previous segment's splitters have been read
    const SsSeg sg = segs[sidx];
    for (uint32_t b = t; b < (uint32_t)SS_NB; b += SS_THREADS) counts[(size_t)sidx * SS_NB + b] = 0u;
    const uint32_t q = ss_splitters(sg.size);
    const uint32_t ns = ss_sample_size(q);
    const uint64_t base = ss_mix(seed ^ (sg.start * 0x9E3779B97F4A7C15ull));
    K x[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {  // every gather in flight before the first LDS store
      const uint32_t j = t + (uint32_t)i * SS_THREADS;
      if (j < ns) {
        const uint64_t h = ss_mix(base + (uint64_t)(j + 1) * 0x9E3779B97F4A7C15ull);
        x[i] = src[sg.start + (((h >> 32) * (uint64_t)sg.size) >> 32)];
      }
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t j = t + (uint32_t)i * SS_THREADS;
      if (j < ns) {
        K y = x[i];
        if constexpr (key_mapped<KK>) y = map_in ? map_key<KK>(y) : y;
        sm.keys[j] = y;
      }
    }
    __syncthreads();
    K mn, mx;
    lds_sort_loaded(sm, ns, mn, mx);
    unsigned char* rec = static_cast<unsigned char*>(spl_rec) + (size_t)sidx * ss_spl_rec_bytes((int)sizeof(K));
    K* rs = reinterpret_cast<K*>(rec);
    auto splitter = [&](uint32_t i) { return sm.keys[(i * q / (uint32_t)SS_P + 1u) * ns / (q + 1u)]; };
    for (uint32_t i = t; i < (uint32_t)SS_P; i += SS_THREADS) rs[i] = splitter(i);
    for (uint32_t k = t + 1; k < 256u; k += SS_THREADS) rs[256 + k] = splitter(ss_tree_sorted_index(k));
    // cell table: cnt[c] = first splitter whose cell is >= c
    const K sbase = splitter(0);
    const int bl = bitlen64((uint64_t)(splitter((uint32_t)SS_P - 1u) - sbase));
    constexpr uint32_t CL = ss_cells_log2((int)sizeof(K)), NC = 1u << CL;
    const uint32_t shift = bl > (int)CL ? (uint32_t)bl - CL : 0u;
    auto first_at = [&](uint32_t cc) {
      uint32_t lo = 0, hi = (uint32_t)SS_P;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (((splitter(mid) - sbase) >> shift) < (K)cc) lo = mid + 1u; else hi = mid;
      }
      return lo;
    };
    uint8_t* cnt = rec + sizeof(K) * 512;
    uint32_t occ = 0;  // most splitters in one cell
    for (uint32_t cc = t; cc <= NC; cc += SS_THREADS) {
      const uint32_t lo = first_at(cc);
      cnt[cc] = (uint8_t)lo;
      if (cc < NC) {
        const uint32_t o = first_at(cc + 1u) - lo;
        occ = o > occ ? o : occ;
      }
    }
    occ = wave_max(occ);
    if (lane_id() == 0) s_occ[t / WAVE] = occ;
    __syncthreads();
    if (t == 0) {
      uint32_t m = 0;
      for (int u = 0; u < SS_THREADS / WAVE; ++u) m = s_occ[u] > m ? s_occ[u] : m;
      reinterpret_cast<uint32_t*>(cnt)[ss_cell_words((int)sizeof(K))] = shift | (m > SS_CELL_MAX ? SS_TREE : 0u);
    }
  }
}

// Clears the status words of the level's tiles.
__global__ __launch_bounds__(256) void k_ss_zero_status(u32x4* __restrict__ status, SsLevelIn lv,
                                                        uint32_t words_per_tile) {
  const uint64_t nvec = (uint64_t)lv.tiles_n() * words_per_tile / 4;
  const u32x4 z = {0u, 0u, 0u, 0u};
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < nvec; i += (uint64_t)gridDim.x * 256) status[i] = z;
}

// ------------------------------------------------------------------ counting
// Each block walks a contiguous range of tiles, classifying keys and
// counting bucket ids in LDS; counts are flushed to the segment's global
// counters whenever the segment changes.
template <int KK>
__global__ __launch_bounds__(SS_THREADS) void k_ss_count(const typename KeyTraits<KK>::K* __restrict__ src, int map_in,
                                                         const SsSeg* __restrict__ segs, SsLevelIn lv,
                                                         uint32_t tile_keys,
                                                         const void* __restrict__ spl,
                                                         uint32_t* __restrict__ counts) {
  using K = typename KeyTraits<KK>::K;
  __shared__ SsCells<K> s_cells;
  __shared__ uint32_t s_cnt[SS_NB];
  const int t = threadIdx.x;
  K base = 0;
  uint32_t shift = 0;
  const uint32_t nsegs = lv.segs_n(), ntiles = lv.tiles_n();
  const uint32_t per = (ntiles + gridDim.x - 1) / gridDim.x;
  const uint32_t t0 = blockIdx.x * per;
  const uint32_t t1 = t0 + per < ntiles ? t0 + per : ntiles;
  int64_t cur = -1;
  for (uint32_t tile = t0; tile < t1; ++tile) {
    const uint32_t sidx = ss_seg_of_tile(segs, nsegs, tile);
    if ((int64_t)sidx != cur) {
      __syncthreads();  // every thread has finished counting the previous tile
      if (cur >= 0) {
        for (int b = t; b < SS_NB; b += SS_THREADS)
          if (s_cnt[b]) add_agent(&counts[(size_t)cur * SS_NB + b], s_cnt[b]);
      }
      __syncthreads();
      for (int b = t; b < SS_NB; b += SS_THREADS) s_cnt[b] = 0;
      shift = ss_cells_load<K, SS_THREADS>(s_cells, spl, sidx);
      cur = sidx;
      __syncthreads();
      base = s_cells.spl[0];
    }
    const SsSeg sg = segs[sidx];
    const uint64_t off = (uint64_t)(tile - sg.first_tile) * tile_keys;
    const uint64_t rem = (uint64_t)sg.size - off;
    const uint32_t cnt = rem < tile_keys ? (uint32_t)rem : tile_keys;
    const K* p = src + sg.start + off;
    constexpr int IPT = sizeof(K) == 4 ? 16 : 8;  // 64-bit keys: registers for eight waves per SIMD
    for (uint32_t b0 = 0; b0 < cnt; b0 += SS_THREADS * IPT) {
      K x[IPT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const uint32_t idx = b0 + (uint32_t)i * SS_THREADS + t;
        x[i] = p[idx < cnt ? idx : cnt - 1];
      }
      // the searches, CS at a time: their LDS reads overlap, while the
      // registers stay few enough for eight waves per SIMD (the scheduler
      // would otherwise interleave all IPT searches and halve the occupancy)
      constexpr int CS = 2;
      uint32_t bk[IPT];
      auto classify_all = [&](auto tree) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
          K y = x[i];
          if constexpr (key_mapped<KK>) y = map_in ? map_key<KK>(y) : y;
          bk[i] = ss_classify<decltype(tree)::value, K>(y, s_cells, base, shift & ~SS_WORD_FLAGS);
          if (i % CS == CS - 1) __builtin_amdgcn_sched_barrier(0);
        }
      };
      if (shift & SS_TREE) classify_all(std::true_type{});
      else classify_all(std::false_type{});
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const bool ok = b0 + (uint32_t)i * SS_THREADS + t < cnt;
        // sorted or run-structured keys put a wave's keys in one bucket,
        // where 64 atomics on one LDS word serialise.  A wave whose first
        // and last lanes share a bucket (a scalar test that random keys
        // almost never pass) adds the lanes of that bucket through its
        // lowest lane; every other key adds 1.  No branch: each lane's
        // increment (0, 1 or the run) masks the one atomic.
        const uint32_t b_first = __builtin_amdgcn_readfirstlane(bk[i]);
        const bool lead = b_first == __builtin_amdgcn_readlane(bk[i], WAVE - 1);
        const bool in_run = lead && ok && bk[i] == b_first;
        const uint64_t run = __ballot(in_run);
        const uint32_t inc = in_run ? (mbcnt(run) == 0 ? popc64(run) : 0u) : (ok ? 1u : 0u);
        if (inc) atomicAdd(&s_cnt[bk[i]], inc);
      }
    }
  }
  __syncthreads();
  if (cur >= 0)
    for (int b = t; b < SS_NB; b += SS_THREADS)
      if (s_cnt[b]) add_agent(&counts[(size_t)cur * SS_NB + b], s_cnt[b]);
}

// ------------------------------------------------------------------ plan
// One block per segment (grid stride): bucket start positions (exclusive
// scan of the counts from the segment start) and the fate of every bucket.
// A bucket of more than SS_CAP / 2 keys stands alone: an equal-key bucket
// is final (copied out unless already in place), an open bucket becomes a
// block-sort item when it has at most SS_CAP keys, else a next-level
// segment.  Smaller buckets of both kinds merge into runs; a run starts at
// a small bucket that follows a standalone one or whose start crosses a
// multiple of SS_CAP / 2, so every run holds fewer than SS_CAP keys.  The
// buckets are ordered ranges, so sorting a run sorts each bucket: a run
// with keys of an open bucket is one block-sort item, a run of equal-key
// buckets only is already sorted and is copied (or left in place).  Merging
// replaces the many tiny items of small segments and of single-key equal
// buckets by items near SS_CAP / 2 keys.  Items and next-level segments
// are numbered with one counter update per segment.
__device__ __forceinline__ bool ss_mask_any(const uint64_t* __restrict__ m, uint32_t lo, uint32_t hi) {
  // any bit of the 512-bit mask m in [lo, hi), lo < hi
  for (uint32_t u = lo / WAVE; u * WAVE < hi; ++u) {
    uint64_t x = m[u];
    if (u == lo / WAVE) x &= ~0ull << (lo % WAVE);
    const uint32_t top = hi - u * WAVE;
    if (top < (uint32_t)WAVE) x &= (1ull << top) - 1ull;
    if (x) return true;
  }
  return false;
}

__global__ __launch_bounds__(SS_NB) void k_ss_plan(const SsSeg* __restrict__ segs, SsLevelIn lv,
                                                   const uint32_t* __restrict__ counts, uint32_t* __restrict__ offs,
                                                   uint32_t dst_buf, int copy_in_place, int eq_out,
                                                   unsigned char* __restrict__ spl, uint32_t rec_bytes,
                                                   uint32_t word_off, SsSeg* __restrict__ next,
                                                   SsItem* __restrict__ items, SsCounters* __restrict__ ctr,
                                                   uint32_t item_cap, uint32_t seg_cap) {
  constexpr int NW = SS_NB / WAVE;
  constexpr uint32_t W = SS_CAP / 2;
  __shared__ uint32_t sm[NW + 1];
  __shared__ uint64_t sm64[NW + 1];
  __shared__ uint32_t s_ex[SS_NB + 1];
  __shared__ uint64_t s_bound[NW], s_open[NW];
  __shared__ unsigned long long s_keys[NW];
  __shared__ uint32_t s_base[2];
  const uint32_t nsegs = lv.segs_n();
  const uint32_t b = threadIdx.x;
  const int w = (int)b / WAVE, lane = lane_id();
  const bool eq_final = dst_buf == SS_BUF_OUT && !copy_in_place;  // equal-key buckets already in place
  for (uint32_t sidx = blockIdx.x; sidx < nsegs; sidx += gridDim.x) {
    const SsSeg sg = segs[sidx];
    const uint32_t c = counts[(size_t)sidx * SS_NB + b];
    uint32_t total;
    const uint32_t ex = block_excl_scan<SS_NB>(c, sm, total);  // ends with a barrier
    offs[(size_t)sidx * SS_NB + b] = ex;  // relative to the segment start
    s_ex[b] = ex;
    if (b == 0) s_ex[SS_NB] = total;
    __syncthreads();
    const bool small = c <= W;
    if (eq_out) {
      // buckets that the scatter writes straight to the output: a bit mask
      // and a flag in the segment's record
      const uint64_t m = __ballot(ss_eq_to_out(b, c));
      unsigned char* rec = spl + (size_t)sidx * rec_bytes;
      uint32_t* mw = reinterpret_cast<uint32_t*>(rec + word_off + 4);
      if (lane == 0) {
        mw[2 * w] = (uint32_t)m;
        mw[2 * w + 1] = (uint32_t)(m >> 32);
        if (m) atomicOr(reinterpret_cast<uint32_t*>(rec + word_off), SS_EQOUT);
      }
    }
    bool start = false;
    if (small) {
      if (b == 0) {
        start = true;
      } else {
        const uint32_t pex = s_ex[b - 1];
        start = ex - pex > W || ex / W != pex / W;
      }
    }
    const uint64_t bm = __ballot(start || !small);
    const uint64_t om = __ballot((b & 1u) == 0u && c > 0u);
    if (lane == 0) { s_bound[w] = bm; s_open[w] = om; }
    __syncthreads();
    // this bucket's items and segments, and its item / segment keys
    uint32_t n_it = 0, n_sg = 0, len = 0, flags = dst_buf << 8;
    uint64_t k_it = 0, k_sg = 0;
    if (start) {
      uint32_t e = SS_NB;  // first boundary after b
      const uint64_t above = lane == WAVE - 1 ? 0ull : bm & (~0ull << (lane + 1));
      if (above) {
        e = (uint32_t)w * WAVE + (uint32_t)__builtin_ctzll(above);
      } else {
        for (int u = w + 1; u < NW; ++u)
          if (s_bound[u]) { e = (uint32_t)u * WAVE + (uint32_t)__builtin_ctzll(s_bound[u]); break; }
      }
      len = s_ex[e] - ex;
      if (len > 0) {
        if (ss_mask_any(s_open, b, e)) {
          n_it = 1;
        } else if (!eq_final) {
          n_it = 1;
          flags |= SS_ITEM_COPY;
        }
      }
    } else if (!small) {
      len = c;
      if (b & 1u) {
        // the scatter wrote it to the output already (eq_out), or it sits
        // in place in the output, or copy items move (and unmap) it there
        if (!eq_final && !(eq_out && ss_eq_to_out(b, c))) n_it = (c + SS_CAP - 1) / SS_CAP;
        flags |= SS_ITEM_COPY;
      } else if (c <= (uint32_t)SS_CAP) {
        n_it = 1;
      } else {
        n_sg = 1;
      }
    }
    if (n_it) k_it = len;
    if (n_sg) k_sg = len;
    // a segment has fewer than 2^32 keys: item and segment keys pack into
    // one 64-bit sum without carries
    const unsigned long long kw = wave_sum((unsigned long long)(k_it | (k_sg << 32)));
    if (lane == 0) s_keys[w] = kw;
    uint64_t tot_pack;
    const uint64_t o_pack = block_excl_scan<SS_NB>((uint64_t)n_it | ((uint64_t)n_sg << 32), sm64, tot_pack);
    if (b == 0) {
      unsigned long long ks = 0;
#pragma unroll
      for (int u = 0; u < NW; ++u) ks += s_keys[u];
      const uint32_t tot_it = (uint32_t)tot_pack, tot_sg = (uint32_t)(tot_pack >> 32);
      s_base[0] = tot_it ? atomicAdd(&ctr->nitems, tot_it) : 0u;
      s_base[1] = tot_sg ? atomicAdd(&ctr->nsegs_next, tot_sg) : 0u;
      if (ks & 0xFFFFFFFFull) atomicAdd(&ctr->item_keys, ks & 0xFFFFFFFFull);
      if (ks >> 32) atomicAdd(&ctr->seg_keys_next, ks >> 32);
    }
    __syncthreads();
    const uint64_t pos = sg.start + ex;
    if (n_it) {
      const uint32_t at = s_base[0] + (uint32_t)o_pack;
      for (uint32_t q = 0; q < n_it; ++q) {
        if (at + q >= item_cap) { atomicOr(&ctr->overflow, 1u); break; }
        SsItem it;
        it.start = pos + (uint64_t)q * SS_CAP;
        it.size = (len - q * SS_CAP) < (uint32_t)SS_CAP ? (len - q * SS_CAP) : (uint32_t)SS_CAP;
        it.flags = flags;
        items[at + q] = it;
      }
    }
    if (n_sg) {
      const uint32_t at = s_base[1] + (uint32_t)(o_pack >> 32);
      if (at >= seg_cap) {
        atomicOr(&ctr->overflow, 2u);
      } else {
        SsSeg ns;
        ns.start = pos;
        ns.size = len;
        ns.first_tile = 0;
        next[at] = ns;
      }
    }
  }
}

// One block: first_tile of every next-level segment (exclusive scan of its
// tile count) and the level's total tile count.
constexpr int SS_TILES_THREADS = 1024;
__global__ __launch_bounds__(SS_TILES_THREADS) void k_ss_tiles(SsSeg* __restrict__ segs, SsCounters* __restrict__ ctr,
                                                               uint32_t tile_keys, uint32_t seg_cap) {
  __shared__ uint32_t sm[SS_TILES_THREADS / WAVE + 1];
  uint32_t nsegs = ctr->nsegs_next;
  if (nsegs > seg_cap) nsegs = seg_cap;
  const uint32_t per = (nsegs + SS_TILES_THREADS - 1) / SS_TILES_THREADS;
  const uint32_t s0 = threadIdx.x * per;
  uint32_t local = 0;
  for (uint32_t i = 0; i < per; ++i)
    if (s0 + i < nsegs) local += (segs[s0 + i].size + tile_keys - 1) / tile_keys;
  uint32_t total;
  uint32_t run = block_excl_scan<SS_TILES_THREADS>(local, sm, total);
  for (uint32_t i = 0; i < per; ++i) {
    if (s0 + i < nsegs) {
      segs[s0 + i].first_tile = run;
      run += (segs[s0 + i].size + tile_keys - 1) / tile_keys;
    }
  }
  if (threadIdx.x == 0) ctr->ntiles_next = total;
}

// ------------------------------------------------------------------ scatter
// Segmented single-pass stable scatter by bucket id (512 ids): the onesweep
// tile machinery with the splitter classifier as the digit, a look-back
// chain per segment and per-segment bucket offsets.  Workgroups take tiles
// in order from an atomic counter until none is left (one tile each when
// the grid has one workgroup per tile); a workgroup only ever waits on
// tiles taken earlier by running workgroups, so any grid size is safe.
template <int KK, bool PAY, int IPT, typename ST, bool PERSIST>
// The persistent form keeps more registers live across its tile loop (212
// VGPRs unbounded); held to four waves per SIMD (two tiles per CU) it spills
// 84 bytes per lane and still runs a graph-captured batch 4 % faster.
__global__ __launch_bounds__(SS_THREADS, PERSIST ? 4 : 1) void k_ss_scatter(SsScatterArgs a) {
  using K = typename KeyTraits<KK>::K;
  constexpr int TILE = SS_THREADS * IPT;
  constexpr int NW = SS_THREADS / WAVE;
  // One LDS region holds in turn the rank state, the dense per-(wave,
  // bucket) position table (written once every count has been read, after
  // the scan's first barrier) and the staged keys with their bucket ids
  // (once every key's tile position is in a register).  Sharing it keeps a
  // u32 tile near 75 KiB, so two tiles fit in a CU's LDS.
  constexpr size_t SLOT_BYTES = sizeof(RankLds<SS_NB>) * NW;
  constexpr size_t KEY_BYTES = sizeof(K) * TILE;
  constexpr size_t STAGE_BYTES = KEY_BYTES + sizeof(uint16_t) * TILE;
  static_assert(sizeof(uint32_t) * NW * SS_NB <= SLOT_BYTES, "position table fits over the slots");
  static_assert(KEY_BYTES % 16 == 0, "bucket ids start aligned after the keys");
  __shared__ __align__(16) unsigned char s_raw[SLOT_BYTES > STAGE_BYTES ? SLOT_BYTES : STAGE_BYTES];
  RankLds<SS_NB>* s_rank = reinterpret_cast<RankLds<SS_NB>*>(s_raw);
  uint32_t(*s_pos)[SS_NB] = reinterpret_cast<uint32_t(*)[SS_NB]>(s_raw);
  K* s_keys = reinterpret_cast<K*>(s_raw);
  uint16_t* s_dig = reinterpret_cast<uint16_t*>(s_raw + KEY_BYTES);
  __shared__ uint32_t s_dadj[SS_NB];  // segment-relative position of tile key j with id b: s_dadj[b] + j
  __shared__ uint32_t s_eqo[SS_NB / 32];  // bit b: bucket b goes straight to the output (ss_eq_to_out)
  __shared__ SsCells<K> s_cells;
  __shared__ uint32_t s_vals[PAY ? TILE : 1];
  __shared__ uint32_t s_scan[NW + 1];
  __shared__ uint32_t s_tile;

  const uint32_t ntiles = a.lv.tiles_n(), nsegs = a.lv.segs_n();
  for (int iter = 0;; ++iter) {
    if (!PERSIST && iter > 0) break;  // one tile per workgroup: no loop to keep registers live across
    // thread and lane ids made opaque per tile: otherwise the compiler hoists
    // the per-item offsets out of the tile loop and holds (spills) them
    uint32_t tv = threadIdx.x;
    asm volatile("" : "+v"(tv));
    const int t = (int)tv, w = t / WAVE, lane = t & (WAVE - 1);
    __syncthreads();  // the previous tile's LDS contents have been consumed
    rank_clear<SS_NB, SS_THREADS>(s_rank, NW);
    if (t == 0) s_tile = add_agent(a.tile_counter, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) break;
    const uint32_t sidx = ss_seg_of_tile(a.segs, nsegs, tile);
    const SsSeg sg = a.segs[sidx];
    const uint64_t off = (uint64_t)(tile - sg.first_tile) * TILE;
    const uint64_t rem = (uint64_t)sg.size - off;
    const uint32_t valid = rem < (uint64_t)TILE ? (uint32_t)rem : (uint32_t)TILE;
    const K* __restrict__ src = (const K*)a.src + sg.start + off;
    const uint32_t* __restrict__ vsrc = PAY ? a.vsrc + sg.start + off : nullptr;

    K k[IPT];
    uint32_t v[IPT];
    uint32_t d[IPT];
    const uint32_t wbase = (uint32_t)w * WAVE * IPT;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      const uint32_t idx = wbase + (uint32_t)i * WAVE + lane;
      k[i] = src[idx < valid ? idx : valid - 1];
      if constexpr (PAY) v[i] = vsrc[idx < valid ? idx : valid - 1];
    }
    // the segment's record after the key loads: its scalar word and its
    // loads overlap theirs
    const uint32_t shift = ss_cells_load<K, SS_THREADS>(s_cells, a.spl, sidx);
    if (shift & SS_EQOUT) {  // uniform: the plan marked buckets for the output
      const uint32_t* mw = ss_eq_mask<K>(a.spl, sidx);
      if (t < SS_NB / 32) s_eqo[t] = mw[t];
    }
    __syncthreads();  // splitters, cell table and output mask in LDS
    const K base = s_cells.spl[0];
    auto classify_all = [&](auto tree) {
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const uint32_t idx = wbase + (uint32_t)i * WAVE + lane;
        K x = k[i];
        if constexpr (key_mapped<KK>) x = a.map_in ? map_key<KK>(x) : x;
        if (idx < valid) {
          k[i] = x;
          d[i] = ss_classify<decltype(tree)::value, K>(x, s_cells, base, shift & ~SS_WORD_FLAGS);
        } else {
          k[i] = ~K(0);
          d[i] = SS_NB - 1;
        }
        // a few searches at a time: interleaving all IPT of them would hold
        // their state in registers beside the tile's keys
        if (i % 2 == 1) __builtin_amdgcn_sched_barrier(0);
      }
    };
    if (shift & SS_TREE) classify_all(std::true_type{});
    else classify_all(std::false_type{});

    uint32_t r[IPT];
    __builtin_amdgcn_sched_barrier(0);
    rank_wave_items<IPT>(d, r, s_rank[w]);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();

    // per-wave exclusive prefixes of bucket t (one bucket per thread)
    static_assert(SS_THREADS == SS_NB, "one bucket id per thread");
    uint32_t cnt = 0, wpre[NW];
#pragma unroll
    for (int u = 0; u < NW; ++u) {
      wpre[u] = cnt;
      cnt += s_rank[u].count[t];
    }
    if (t == SS_NB - 1) cnt -= (uint32_t)TILE - valid;  // padding: last id, sorted last
    uint32_t total;
    const uint32_t tstart = block_excl_scan<SS_THREADS>(cnt, s_scan, total);
    // dense table of tile positions: one LDS read per key below
#pragma unroll
    for (int u = 0; u < NW; ++u) s_pos[u][t] = wpre[u] + tstart;
    const uint64_t excl = lookback<SS_NB, ST>((ST*)a.status, tile, sg.first_tile, (uint32_t)t, cnt);
    s_dadj[t] = a.offs[(size_t)sidx * SS_NB + t] + (uint32_t)excl - tstart;  // modulo 2^32
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) r[i] += s_pos[w][d[i]];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
      if (r[i] < (uint32_t)TILE) {
        s_keys[r[i]] = k[i];
        if constexpr (PAY) s_vals[r[i]] = v[i];
        s_dig[r[i]] = (uint16_t)d[i];
      }
    }
    __syncthreads();

    K* __restrict__ dst = (K*)a.dst;
    auto put = [&](uint32_t j, K x, uint32_t rel) {
      if (rel >= sg.size) return;  // unreachable with consistent counts
      const uint64_t o = sg.start + rel;
      dst[o] = x;
      if constexpr (PAY) a.vdst[o] = s_vals[j];
    };
    if (shift & SS_EQOUT) {
      // some bucket of equal keys goes to the output (uniform over the
      // workgroup): one key at a time, each with its destination buffer
      K* __restrict__ kout = (K*)a.out;
#pragma unroll 4
      for (uint32_t j = t; j < valid; j += SS_THREADS) {
        K x = s_keys[j];
        const uint32_t dg = s_dig[j];
        const uint32_t rel = s_dadj[dg] + j;
        if (rel >= sg.size) continue;  // unreachable with consistent counts
        const uint64_t o = sg.start + rel;
        if ((s_eqo[dg >> 5] >> (dg & 31u)) & 1u) {
          if constexpr (key_mapped<KK>) x = unmap_key<KK>(x);
          kout[o] = x;
          if constexpr (PAY) a.vout[o] = s_vals[j];
        } else {
          dst[o] = x;
          if constexpr (PAY) a.vdst[o] = s_vals[j];
        }
      }
    } else if (valid == (uint32_t)TILE) {
      // full tile: all LDS reads first, then the stores
      K x[IPT];
      uint32_t rel[IPT];
#pragma unroll
      for (int i = 0; i < IPT; ++i) {
        const uint32_t j = (uint32_t)(t + i * SS_THREADS);
        x[i] = s_keys[j];
        rel[i] = s_dig[j];
      }
#pragma unroll
      for (int i = 0; i < IPT; ++i) rel[i] = s_dadj[rel[i]] + (uint32_t)(t + i * SS_THREADS);
#pragma unroll
      for (int i = 0; i < IPT; ++i) put((uint32_t)(t + i * SS_THREADS), x[i], rel[i]);
    } else {
      for (uint32_t j = t; j < valid; j += SS_THREADS) put(j, s_keys[j], s_dadj[s_dig[j]] + j);
    }
  }
}

// ------------------------------------------------------------------ block sort
// COPY items move (and unmap) keys.  SORT items (at most SS_CAP keys) are
// loaded into LDS and sorted by lds_sort_loaded.
template <int KK, bool PAY>
__device__ __forceinline__ void ss_block_item(const SsBlockArgs& a, BlockSortSmem<typename KeyTraits<KK>::K, PAY>& sm,
                                              uint32_t item) {
  using K = typename KeyTraits<KK>::K;
  const int t = threadIdx.x;
  K* __restrict__ dst = (K*)a.kout;
  const SsItem it = a.items[item];
  const uint32_t buf = (it.flags >> 8) & 0xFFu;
  const K* __restrict__ src = (const K*)(buf == SS_BUF_IN ? a.kin : (buf == SS_BUF_OUT ? a.kout : a.ktmp));
  const uint32_t* __restrict__ vsrc = buf == SS_BUF_IN ? a.vin : (buf == SS_BUF_OUT ? a.vout : a.vtmp);
  const bool raw = buf == SS_BUF_IN;
  const uint64_t base = it.start;
  const uint32_t size = it.size;
  if (it.flags & SS_ITEM_COPY) {
    // groups of CI loads in flight per thread, then their stores
    constexpr int CI = 16;
    for (uint32_t j0 = 0; j0 < size; j0 += SS_THREADS * CI) {
      K x[CI];
      uint32_t v[CI];
#pragma unroll
      for (int i = 0; i < CI; ++i) {
        const uint32_t j = j0 + t + (uint32_t)i * SS_THREADS;
        if (j < size) {
          x[i] = src[base + j];
          if constexpr (PAY) v[i] = vsrc[base + j];
        }
      }
#pragma unroll
      for (int i = 0; i < CI; ++i) {
        const uint32_t j = j0 + t + (uint32_t)i * SS_THREADS;
        if (j < size) {
          K y = x[i];
          if constexpr (key_mapped<KK>) y = raw ? y : unmap_key<KK>(y);
          dst[base + j] = y;
          if constexpr (PAY) a.vout[base + j] = v[i];
        }
      }
    }
    return;
  }
  lds_load_mapped<KK, PAY>(sm, src + base, PAY ? vsrc + base : nullptr, size, raw);
  K mn, mx;
  lds_sort_loaded(sm, size, mn, mx);
  for (uint32_t j = t; j < size; j += SS_THREADS) {
    K x = sm.keys[j];
    if constexpr (key_mapped<KK>) x = unmap_key<KK>(x);
    dst[base + j] = x;
    if constexpr (PAY) a.vout[base + j] = sm.vals[j];
  }
}

// One item per workgroup (host-driven levels), or workgroups striding over
// the items whose count the device holds (device-driven levels).
template <int KK, bool PAY, bool PERSIST>
__global__ __launch_bounds__(SS_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_ss_block(SsBlockArgs a) {
  using K = typename KeyTraits<KK>::K;
  __shared__ BlockSortSmem<K, PAY> sm;
  if constexpr (!PERSIST) {
    if (blockIdx.x < a.nitems) ss_block_item<KK, PAY>(a, sm, blockIdx.x);
  } else {
    uint32_t nitems = a.lvl ? a.lvl->nitems : a.nitems;
    nitems = nitems < a.item_cap ? nitems : a.item_cap;
    for (uint32_t item = blockIdx.x; item < nitems; item += gridDim.x) {
      __syncthreads();  // the previous item's LDS contents have been stored
      ss_block_item<KK, PAY>(a, sm, item);
    }
  }
}

// ------------------------------------------------------------------ launchers
hipError_t launch_ss_init(SsSeg* segs, SsItem* items, uint64_t n, SsCounters* ctr, uint32_t* tilectr, int levels,
                          hipStream_t s) {
  if (levels < 0 || levels > SS_MAX_LEVELS || (segs && !items)) return hipErrorInvalidValue;
  k_ss_init<<<1, 256, 0, s>>>(segs, items, n, reinterpret_cast<uint32_t*>(ctr),
                              (uint32_t)(sizeof(SsCounters) / 4 * levels), tilectr, (uint32_t)levels);
  return hipGetLastError();
}

hipError_t launch_ss_sample(int kk, const void* src, int map_in, const SsSeg* segs, const SsLevelIn& lv, void* spl,
                            uint32_t* counts, uint64_t seed, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if ((uint32_t)nblocks > MAX_GRID_BLOCKS) nblocks = (int)MAX_GRID_BLOCKS;  // the kernel strides over segments
  switch (kk) {
    case KK_U32: k_ss_sample<KK_U32><<<nblocks, SS_THREADS, 0, s>>>((const uint32_t*)src, map_in, segs, lv, spl, counts, seed); break;
    case KK_U64: k_ss_sample<KK_U64><<<nblocks, SS_THREADS, 0, s>>>((const uint64_t*)src, map_in, segs, lv, spl, counts, seed); break;
    case KK_F32: k_ss_sample<KK_F32><<<nblocks, SS_THREADS, 0, s>>>((const uint32_t*)src, map_in, segs, lv, spl, counts, seed); break;
    case KK_I32: k_ss_sample<KK_I32><<<nblocks, SS_THREADS, 0, s>>>((const uint32_t*)src, map_in, segs, lv, spl, counts, seed); break;
    case KK_F64: k_ss_sample<KK_F64><<<nblocks, SS_THREADS, 0, s>>>((const uint64_t*)src, map_in, segs, lv, spl, counts, seed); break;
    case KK_I64: k_ss_sample<KK_I64><<<nblocks, SS_THREADS, 0, s>>>((const uint64_t*)src, map_in, segs, lv, spl, counts, seed); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ss_zero_status(void* status, const SsLevelIn& lv, uint32_t words_per_tile, hipStream_t s) {
  // host-driven: exact grid; device-driven: a fixed grid that strides
  uint64_t nvec = lv.in ? (uint64_t)lv.tile_cap * words_per_tile / 4 : (uint64_t)lv.ntiles * words_per_tile / 4;
  if (nvec == 0) return hipSuccess;
  const uint64_t nb = (nvec + 255) / 256;
  const uint32_t grid = (uint32_t)(nb < 4096 ? nb : 4096);
  k_ss_zero_status<<<grid, 256, 0, s>>>(static_cast<u32x4*>(status), lv, words_per_tile);
  return hipGetLastError();
}

hipError_t launch_ss_count(int kk, const void* src, int map_in, const SsSeg* segs, const SsLevelIn& lv,
                           const void* spl, uint32_t* counts, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  const uint32_t tk = (uint32_t)ss_tile(key_bytes_of(kk));
  switch (kk) {
    case KK_U32: k_ss_count<KK_U32><<<nblocks, SS_THREADS, 0, s>>>((const uint32_t*)src, map_in, segs, lv, tk, spl, counts); break;
    case KK_U64: k_ss_count<KK_U64><<<nblocks, SS_THREADS, 0, s>>>((const uint64_t*)src, map_in, segs, lv, tk, spl, counts); break;
    case KK_F32: k_ss_count<KK_F32><<<nblocks, SS_THREADS, 0, s>>>((const uint32_t*)src, map_in, segs, lv, tk, spl, counts); break;
    case KK_I32: k_ss_count<KK_I32><<<nblocks, SS_THREADS, 0, s>>>((const uint32_t*)src, map_in, segs, lv, tk, spl, counts); break;
    case KK_F64: k_ss_count<KK_F64><<<nblocks, SS_THREADS, 0, s>>>((const uint64_t*)src, map_in, segs, lv, tk, spl, counts); break;
    case KK_I64: k_ss_count<KK_I64><<<nblocks, SS_THREADS, 0, s>>>((const uint64_t*)src, map_in, segs, lv, tk, spl, counts); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ss_plan(const SsSeg* segs, const SsLevelIn& lv, const uint32_t* counts, uint32_t* offs,
                          uint32_t dst_buf, int copy_in_place, int eq_out, void* spl, int key_bytes, SsSeg* next,
                          SsItem* items, SsCounters* ctr, uint32_t item_cap, uint32_t seg_cap, int nblocks,
                          hipStream_t s) {
  if (key_bytes != 4 && key_bytes != 8) return hipErrorInvalidValue;
  if (nblocks <= 0) return hipSuccess;
  if ((uint32_t)nblocks > MAX_GRID_BLOCKS) nblocks = (int)MAX_GRID_BLOCKS;  // the kernel strides over segments
  k_ss_plan<<<nblocks, SS_NB, 0, s>>>(segs, lv, counts, offs, dst_buf, copy_in_place, eq_out, static_cast<unsigned char*>(spl),
                                      (uint32_t)ss_spl_rec_bytes(key_bytes), (uint32_t)ss_word_offset(key_bytes), next, items, ctr, item_cap,
                                      seg_cap);
  return hipGetLastError();
}

hipError_t launch_ss_tiles(SsSeg* segs, SsCounters* ctr, uint32_t tile_keys, uint32_t seg_cap, hipStream_t s) {
  k_ss_tiles<<<1, SS_TILES_THREADS, 0, s>>>(segs, ctr, tile_keys, seg_cap);
  return hipGetLastError();
}

template <int KK, bool PAY, typename ST>
static const void* scatter_fn() {
  constexpr int IPT = sizeof(typename KeyTraits<KK>::K) == 4 ? SS_IPT32 : SS_IPT64;
  return reinterpret_cast<const void*>(&k_ss_scatter<KK, PAY, IPT, ST, true>);
}

template <int KK, bool PAY, bool PERSIST>
static hipError_t scatter_kk(const SsScatterArgs& a, uint32_t grid, hipStream_t s) {
  constexpr int IPT = sizeof(typename KeyTraits<KK>::K) == 4 ? SS_IPT32 : SS_IPT64;
  if (a.max_seg < STATUS32_MAX_N)
    k_ss_scatter<KK, PAY, IPT, uint32_t, PERSIST><<<grid, SS_THREADS, 0, s>>>(a);
  else
    k_ss_scatter<KK, PAY, IPT, uint64_t, PERSIST><<<grid, SS_THREADS, 0, s>>>(a);
  return hipGetLastError();
}

template <bool PERSIST>
static hipError_t scatter_any(int kk, int with_vals, const SsScatterArgs& a, uint32_t grid, hipStream_t s) {
  switch (kk * 2 + (with_vals ? 1 : 0)) {
    case KK_U32 * 2: return scatter_kk<KK_U32, false, PERSIST>(a, grid, s);
    case KK_U32 * 2 + 1: return scatter_kk<KK_U32, true, PERSIST>(a, grid, s);
    case KK_U64 * 2: return scatter_kk<KK_U64, false, PERSIST>(a, grid, s);
    case KK_U64 * 2 + 1: return scatter_kk<KK_U64, true, PERSIST>(a, grid, s);
    case KK_F32 * 2: return scatter_kk<KK_F32, false, PERSIST>(a, grid, s);
    case KK_I32 * 2: return scatter_kk<KK_I32, false, PERSIST>(a, grid, s);
    case KK_F32 * 2 + 1: return scatter_kk<KK_F32, true, PERSIST>(a, grid, s);
    case KK_I32 * 2 + 1: return scatter_kk<KK_I32, true, PERSIST>(a, grid, s);
    case KK_F64 * 2: return scatter_kk<KK_F64, false, PERSIST>(a, grid, s);
    case KK_I64 * 2: return scatter_kk<KK_I64, false, PERSIST>(a, grid, s);
    case KK_F64 * 2 + 1: return scatter_kk<KK_F64, true, PERSIST>(a, grid, s);
    case KK_I64 * 2 + 1: return scatter_kk<KK_I64, true, PERSIST>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ss_scatter(int kk, int with_vals, const SsScatterArgs& a, uint32_t nblocks, hipStream_t s) {
  if (nblocks) {
    if (!grid_fits(nblocks, SS_THREADS)) return hipErrorInvalidConfiguration;
    return scatter_any<true>(kk, with_vals, a, nblocks, s);
  }
  if (a.lv.ntiles == 0) return hipSuccess;
  if (a.lv.ntiles > MAX_GRID_BLOCKS)  // one workgroup per tile would overflow the dispatch
    return scatter_any<true>(kk, with_vals, a, MAX_GRID_BLOCKS, s);
  return scatter_any<false>(kk, with_vals, a, a.lv.ntiles, s);
}

template <bool PERSIST>
static hipError_t block_any(int kk, int with_vals, const SsBlockArgs& a, uint32_t grid, hipStream_t s) {
  switch (kk * 2 + (with_vals ? 1 : 0)) {
    case KK_U32 * 2: k_ss_block<KK_U32, false, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_U32 * 2 + 1: k_ss_block<KK_U32, true, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_U64 * 2: k_ss_block<KK_U64, false, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_U64 * 2 + 1: k_ss_block<KK_U64, true, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_F32 * 2: k_ss_block<KK_F32, false, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_I32 * 2: k_ss_block<KK_I32, false, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_F32 * 2 + 1: k_ss_block<KK_F32, true, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_I32 * 2 + 1: k_ss_block<KK_I32, true, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_F64 * 2: k_ss_block<KK_F64, false, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_I64 * 2: k_ss_block<KK_I64, false, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_F64 * 2 + 1: k_ss_block<KK_F64, true, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    case KK_I64 * 2 + 1: k_ss_block<KK_I64, true, PERSIST><<<grid, SS_THREADS, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ss_block(int kk, int with_vals, const SsBlockArgs& a, uint32_t nblocks, hipStream_t s) {
  if (nblocks) {
    if (!grid_fits(nblocks, SS_THREADS)) return hipErrorInvalidConfiguration;
    return block_any<true>(kk, with_vals, a, nblocks, s);
  }
  if (a.nitems == 0) return hipSuccess;
  if (a.nitems > MAX_GRID_BLOCKS) {  // one workgroup per item would overflow the dispatch
    SsBlockArgs b = a;
    b.lvl = nullptr;
    b.item_cap = a.nitems;
    return block_any<true>(kk, with_vals, b, MAX_GRID_BLOCKS, s);
  }
  return block_any<false>(kk, with_vals, a, a.nitems, s);
}

static uint32_t resident(const void* fn, int threads, uint32_t cu_count) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  return (uint32_t)per_cu * (cu_count ? cu_count : 1);
}

uint32_t ss_scatter_resident(int kk, int with_vals, uint64_t max_seg, uint32_t cu_count) {
  const bool s32 = max_seg < STATUS32_MAX_N;
  const void* fn = nullptr;
  switch (kk * 2 + (with_vals ? 1 : 0)) {
    case KK_U32 * 2: fn = s32 ? scatter_fn<KK_U32, false, uint32_t>() : scatter_fn<KK_U32, false, uint64_t>(); break;
    case KK_U32 * 2 + 1: fn = s32 ? scatter_fn<KK_U32, true, uint32_t>() : scatter_fn<KK_U32, true, uint64_t>(); break;
    case KK_U64 * 2: fn = s32 ? scatter_fn<KK_U64, false, uint32_t>() : scatter_fn<KK_U64, false, uint64_t>(); break;
    case KK_U64 * 2 + 1: fn = s32 ? scatter_fn<KK_U64, true, uint32_t>() : scatter_fn<KK_U64, true, uint64_t>(); break;
    case KK_F32 * 2: fn = s32 ? scatter_fn<KK_F32, false, uint32_t>() : scatter_fn<KK_F32, false, uint64_t>(); break;
    case KK_I32 * 2: fn = s32 ? scatter_fn<KK_I32, false, uint32_t>() : scatter_fn<KK_I32, false, uint64_t>(); break;
    case KK_F32 * 2 + 1: fn = s32 ? scatter_fn<KK_F32, true, uint32_t>() : scatter_fn<KK_F32, true, uint64_t>(); break;
    case KK_I32 * 2 + 1: fn = s32 ? scatter_fn<KK_I32, true, uint32_t>() : scatter_fn<KK_I32, true, uint64_t>(); break;
    case KK_F64 * 2: fn = s32 ? scatter_fn<KK_F64, false, uint32_t>() : scatter_fn<KK_F64, false, uint64_t>(); break;
    case KK_I64 * 2: fn = s32 ? scatter_fn<KK_I64, false, uint32_t>() : scatter_fn<KK_I64, false, uint64_t>(); break;
    case KK_I64 * 2 + 1: fn = s32 ? scatter_fn<KK_I64, true, uint32_t>() : scatter_fn<KK_I64, true, uint64_t>(); break;
    default: fn = s32 ? scatter_fn<KK_F64, true, uint32_t>() : scatter_fn<KK_F64, true, uint64_t>(); break;
  }
  return resident(fn, SS_THREADS, cu_count);
}

uint32_t ss_block_resident(int kk, int with_vals, uint32_t cu_count) {
  const void* fn = nullptr;
  switch (kk * 2 + (with_vals ? 1 : 0)) {
    case KK_U32 * 2: fn = reinterpret_cast<const void*>(&k_ss_block<KK_U32, false, true>); break;
    case KK_U32 * 2 + 1: fn = reinterpret_cast<const void*>(&k_ss_block<KK_U32, true, true>); break;
    case KK_U64 * 2: fn = reinterpret_cast<const void*>(&k_ss_block<KK_U64, false, true>); break;
    case KK_U64 * 2 + 1: fn = reinterpret_cast<const void*>(&k_ss_block<KK_U64, true, true>); break;
    case KK_F32 * 2: fn = reinterpret_cast<const void*>(&k_ss_block<KK_F32, false, true>); break;
    case KK_I32 * 2: fn = reinterpret_cast<const void*>(&k_ss_block<KK_I32, false, true>); break;
    case KK_F32 * 2 + 1: fn = reinterpret_cast<const void*>(&k_ss_block<KK_F32, true, true>); break;
    case KK_I32 * 2 + 1: fn = reinterpret_cast<const void*>(&k_ss_block<KK_I32, true, true>); break;
    case KK_F64 * 2: fn = reinterpret_cast<const void*>(&k_ss_block<KK_F64, false, true>); break;
    case KK_I64 * 2: fn = reinterpret_cast<const void*>(&k_ss_block<KK_I64, false, true>); break;
    case KK_I64 * 2 + 1: fn = reinterpret_cast<const void*>(&k_ss_block<KK_I64, true, true>); break;
    default: fn = reinterpret_cast<const void*>(&k_ss_block<KK_F64, true, true>); break;
  }
  return resident(fn, SS_THREADS, cu_count);
}

}  // namespace ahs
