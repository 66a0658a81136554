// Host-side launchers of the gfx950 kernels and the small structures they
// share with the host dispatcher.  Every launcher enqueues on `s` and
// returns the hipError_t of the launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ahs {

// Key kinds: the dtype enum of the ABI, as template parameters.
enum KeyKind : int { KK_U32 = 0, KK_U64 = 1, KK_F32 = 2, KK_F64 = 3, KK_I32 = 4, KK_I64 = 5 };
constexpr int NUM_KEY_KINDS = 6;  // tables indexed by the key kind have this many rows
inline int key_bytes_of(int kk) { return (kk == KK_U64 || kk == KK_F64 || kk == KK_I64) ? 8 : 4; }

// Bit length of a 64-bit value (0 for 0).
__host__ __device__ __forceinline__ int bitlen64(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

// Device copy of the feature vector; same layout as ahs_feature_vector.
struct DevFeatures {
  uint64_t n, min_key, max_key, span, nan_count;
  uint32_t shift, nbins, exact, reserved;
  double entropy_bits, entropy_ratio;
};

struct MinMaxPartial {
  uint64_t mn, mx, nan;
  uint64_t pad;
};

// A dispatch counts work-items in 32 bits: grid x block must stay below
// 2^32.  Kernels whose work can exceed this take a grid stride, and the host
// caps their grids at MAX_GRID_BLOCKS.
constexpr uint32_t MAX_GRID_BLOCKS = 1u << 22;
inline bool grid_fits(uint64_t blocks, uint32_t threads) { return blocks * (uint64_t)threads < (1ull << 32); }

// Launch-geometry constants used by both the host planner and the kernels.
constexpr int HIST_SMALL_MAX_BINS = 8192;      // u32 LDS bins
constexpr int HIST_LARGE_WORDS = 32768;        // 65,536 packed u16 bins
constexpr int MINMAX_THREADS = 256;
constexpr int HIST_SMALL_THREADS = 256;
constexpr int HIST_LARGE_THREADS = 1024;
constexpr int DIGIT_HIST_THREADS = 256;
constexpr int EXPAND_THREADS = 256;
constexpr int EXPAND_TILE = EXPAND_THREADS * 4 * 8;   // positions per block

// Onesweep tile shapes: 512 threads (8 waves) per tile, two tiles resident
// per CU (at most 128 VGPRs and 80 KiB of LDS each).
#ifndef AHS_OS_THREADS
#define AHS_OS_THREADS 512
#endif
constexpr int OS_THREADS = AHS_OS_THREADS;
constexpr int OS_WAVES = OS_THREADS / 64;
// Keys per thread of a onesweep tile (compile-time tunable): the largest
// that keep two tiles per CU.  Larger tiles shorten the look-back chain and
// lengthen the runs of consecutive addresses the scatter writes (one run
// per digit and tile: at 48 keys per run a plain run-copy of 2^28 u32 keys
// reaches 4.0 TB/s, at 96 keys 5.1 TB/s).  Measured on 2^28 u32 / 2^27 u64
// passes: 32 keys per thread 0.690 ms against 0.744 ms at 24; 18 for u64
// keys and for u32 keys with payload; 12 for u64 with payload (14 would
// leave one tile per CU).  One tile per CU (1,024 threads or an 80 KiB+
// tile) loses the overlap of one tile's memory phases with the other's
// ranking and is slower at any tile size tried.
#ifndef AHS_OS_IPT32
#define AHS_OS_IPT32 32
#endif
#ifndef AHS_OS_IPT64
#define AHS_OS_IPT64 18
#endif
#ifndef AHS_OS_IPT32P
#define AHS_OS_IPT32P 18
#endif
#ifndef AHS_OS_IPT64P
#define AHS_OS_IPT64P 12
#endif
constexpr int OS_IPT32 = AHS_OS_IPT32, OS_IPT64 = AHS_OS_IPT64;
constexpr int OS_IPT32P = AHS_OS_IPT32P, OS_IPT64P = AHS_OS_IPT64P;
inline int os_items(int key_bytes, bool pay) {
  return key_bytes == 4 ? (pay ? OS_IPT32P : OS_IPT32) : (pay ? OS_IPT64P : OS_IPT64);
}
inline int os_tile(int key_bytes, bool pay) { return OS_THREADS * os_items(key_bytes, pay); }

// Look-back status words are 32-bit below this many keys, 64-bit above.
constexpr uint64_t STATUS32_MAX_N = 1ull << 30;
inline size_t status_word_bytes(uint64_t n) { return n < STATUS32_MAX_N ? 4 : 8; }

// ---------------------------------------------------------------- features
// Histogram plan for the AUTO feature step without a host round trip: the
// min/max kernel derives it from the span and the thresholds and leaves it
// in DevFeatures::reserved; the histogram, reduce and digit kernels given a
// `plan` pointer read their sizes from the device and skip what the plan
// does not need.
constexpr uint32_t PLAN_ON = 1u << 31;
constexpr uint32_t PLAN_LARGE = 1u;  // the 65,536-bin packed histogram (else the exact small one)
constexpr uint32_t PLAN_SKIP = 2u;   // no histogram needed
constexpr uint32_t PLAN_FUSED = 4u;  // the exact histogram is the min/max pass's modulo counts, rotated by min
inline __host__ __device__ int plan_digits(uint32_t plan) { return (int)((plan >> 4) & 15u); }
// Of those digits, the ones the fused histogram counts per key: digit p
// (bits 8p .. 8p+7 of key - min) with 8p >= shift is (bin >> (8p - shift))
// & 255 for the key's histogram bin, so its counts follow from the reduced
// histogram; only the digits below the shift need a count per key.
inline __host__ __device__ int plan_fused_digits(uint32_t plan, uint32_t shift) {
  const int below = (int)((shift + 7u) / 8u);
  return plan_digits(plan) < below ? plan_digits(plan) : below;
}
struct FeaturePlanCfg {
  uint64_t kcount_minus1, k_radix, n_small;
  uint32_t enabled, model, want_hist;
  uint32_t fused;  // the min/max pass also counted every key by its mapped value modulo HIST_SMALL_MAX_BINS
};
constexpr int HRED_MAX_BLOCKS = 1024;  // reduce blocks covering 65,536 bins

// With mod_partials (AUTO only) every block also counts its non-NaN keys
// by mapped value modulo HIST_SMALL_MAX_BINS into mod_partials[block][.]:
// when the span turns out below HIST_SMALL_MAX_BINS that is the exact
// histogram of key - min rotated by min, and the plan marks it PLAN_FUSED.
// With a plan and corr set, a plan for the packed 65,536-bin histogram also
// zeroes its 65,536 correction words.
hipError_t launch_minmax(int kk, const void* keys, uint64_t n, MinMaxPartial* partials, int nblocks,
                         DevFeatures* df, hipStream_t s, const FeaturePlanCfg* plan_cfg = nullptr,
                         uint32_t* mod_partials = nullptr, uint32_t* corr = nullptr);
hipError_t launch_hist_small(int kk, const void* keys, uint64_t n, uint64_t kmin, uint32_t shift,
                             uint32_t nbins, uint32_t* partials, int nblocks, hipStream_t s,
                             const DevFeatures* plan = nullptr);
hipError_t launch_hist_large(int kk, const void* keys, uint64_t n, uint64_t kmin, uint32_t shift,
                             uint32_t* partials, uint32_t* corr, int nblocks, int ndig,
                             uint32_t* digit_partials, hipStream_t s, const DevFeatures* plan = nullptr);
// With a plan: ngroups is the small histogram's block count and
// ngroups_large the large one's (the same when the planned large kernel
// counted the small histogram too); the grid covers 65,536 bins.
hipError_t launch_hist_reduce(const uint32_t* partials, int ngroups, uint32_t nbins, int large,
                              const uint32_t* corr, uint32_t* hist_out, uint64_t n, double* hpart,
                              int* nparts_out, hipStream_t s, const DevFeatures* plan = nullptr,
                              int ngroups_large = 0, int ngroups_fused = 0);
hipError_t launch_entropy_final(const double* hpart, int nparts, DevFeatures* df, hipStream_t s);

// ---------------------------------------------------------------- counting
hipError_t launch_scan_bins(const uint32_t* hist, uint32_t nbins, uint32_t* offsets, hipStream_t s);
hipError_t launch_expand(int kk, const uint32_t* offsets, uint32_t nbins, uint64_t kmin, void* out,
                         uint64_t n, hipStream_t s);

// ---------------------------------------------------------------- radix
hipError_t launch_digit_hist(int kk, const void* keys, uint64_t n, uint64_t kmin, int ndig,
                             uint32_t* digit_partials, int nblocks, hipStream_t s);
// Sums per-block digit counts into counts[ndig][256] and their exclusive
// scans into offsets[ndig][256].  With hpart (nparts entropy partials of the
// histogram reduce) it also finishes the entropy into df, as
// launch_entropy_final would.
hipError_t launch_digit_reduce(const uint32_t* digit_partials, const uint32_t* hist, int nblocks, int ndig,
                               uint32_t* counts, uint32_t* offsets, hipStream_t s,
                               const DevFeatures* plan = nullptr, const double* hpart = nullptr, int nparts = 0,
                               DevFeatures* df = nullptr);
hipError_t launch_fill_u64(uint64_t* p, uint64_t count, uint64_t value, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint64_t count, uint32_t value, hipStream_t s);

struct OnesweepArgs {
  const void* src;
  void* dst;
  const uint32_t* vsrc;
  uint32_t* vdst;
  uint64_t n;
  uint64_t kmin;
  uint32_t digit_shift;   // digit = ((key - kmin) >> digit_shift) & 255
  uint32_t map_in;        // keys in src are raw (apply the float map)
  uint32_t unmap_out;     // write raw keys to dst (apply the inverse map)
  const uint32_t* digit_offsets;  // [256] global exclusive offsets of this pass
  void* status;           // [tiles][256] words of status_word_bytes(n), zero before the launch
  uint32_t* tile_counter; // zero before the launch
};
hipError_t launch_onesweep(int kk, int with_vals, const OnesweepArgs& a, hipStream_t s);

// ---------------------------------------------------------------- small
hipError_t launch_small_sort(int kk, const void* src, void* dst, const uint32_t* vsrc, uint32_t* vdst,
                             uint32_t n, hipStream_t s);
constexpr int SMALL_SORT_MAX = 1024;

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace ahs
