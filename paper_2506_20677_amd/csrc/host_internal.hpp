// Internal host-side state: the context, the workspace layout and the
// helpers the strategy drivers share.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "ahs.h"
#include "kernels.hpp"

struct ahs_context {
  static constexpr size_t PINNED_BYTES = 1 << 20;
  int device = 0;
  uint32_t cu_count = 0;
  std::string device_name;
  std::string last_error;
  const ahs_model* model = nullptr;
  void* pinned = nullptr;  // host staging for small device-to-host reads
  void* static_scratch = nullptr;  // device address of this device's ahs_sort_static scratch

  // per-kernel event timing
  struct Rec {
    std::string name;
    double bytes = 0.0;  // algorithmic HBM bytes of the launch
    hipEvent_t a = nullptr, b = nullptr;
  };
  struct Total {
    uint64_t launches = 0;
    double ms = 0.0, bytes = 0.0;
  };
  bool profiling = false;
  bool capturing = false;  // a stream capture is recording: no timing events
  std::vector<Rec> pending;
  std::vector<hipEvent_t> event_pool;
  std::map<std::string, Total> totals;

  // Batched sort: LDS kernel variant (0..3, capacity 1024 << v) per key
  // type, payload flag and size class; set by the autotuner.
  int seg_variant[ahs::NUM_KEY_KINDS][2][4] = {{{0, 1, 2, 3}, {0, 1, 2, 3}}, {{0, 1, 2, 3}, {0, 1, 2, 3}},
                                          {{0, 1, 2, 3}, {0, 1, 2, 3}}, {{0, 1, 2, 3}, {0, 1, 2, 3}},
                                          {{0, 1, 2, 3}, {0, 1, 2, 3}}, {{0, 1, 2, 3}, {0, 1, 2, 3}}};
  static_assert(ahs::NUM_KEY_KINDS == 6, "one row of defaults per key kind");
  // Batched sort: tile variant (0 small, 1 large) of the segmented radix
  // passes per key type and payload flag; set by the autotuner.
  int seg_radix_variant[ahs::NUM_KEY_KINDS][2] = {{1, 1}, {1, 1}, {1, 1}, {1, 1}, {1, 1}, {1, 1}};

  ~ahs_context();
  ahs_status fail(ahs_status s, const char* fmt, ...);
  ahs_status check(hipError_t e, const char* what);
  hipEvent_t take_event();
  void prof_begin(const char* name, hipStream_t s, double bytes);
  void prof_end(hipStream_t s);
  // Sets the algorithmic bytes of the latest pending launch record named
  // `name` (launches whose work the device decides, known after a read-back).
  void prof_set_last_bytes(const char* name, double bytes);
  void prof_collect();
};

#define AHS_TRY(expr)                    \
  do {                                   \
    ahs_status st__ = (expr);            \
    if (st__ != AHS_OK) return st__;     \
  } while (0)

#define AHS_HIP(j, call, what) AHS_TRY((j).ctx->check((call), (what)))

namespace ahs {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint64_t clamp_u64(uint64_t x, uint64_t lo, uint64_t hi) { return x < lo ? lo : (x > hi ? hi : x); }

// Grid sizes depend only on n, so the workspace size is data-independent.
// (min/max streams fastest with about two workgroups per CU: 512 of 256
// threads measured 5.4 TB/s on 1 GiB, 2,048 only 3.8 TB/s)
inline int minmax_blocks(uint64_t n) { return (int)clamp_u64(ceil_div(n, 1u << 19), 1, 512); }
inline int hist_small_blocks(uint64_t n) { return (int)clamp_u64(ceil_div(n, 65536), 1, 512); }
// One workgroup of the packed 65,536-bin histogram per 2^14 keys, at most
// one per CU (its 128 KiB of LDS allows one): every CU takes part from 2^22
// keys up, while each workgroup's fixed cost (clearing and flushing its bins)
// stays below the time of its keys on smaller arrays.
inline int hist_large_blocks(uint64_t n) { return (int)clamp_u64(ceil_div(n, 1u << 14), 1, 256); }
inline int digit_hist_blocks(uint64_t n) { return (int)clamp_u64(ceil_div(n, 65536), 1, 1024); }

struct Layout {
  size_t df = 0, mm = 0, hpart = 0, hist_parts = 0, corr = 0, hist = 0, offs = 0;
  size_t dparts = 0, dcounts = 0, doffs = 0, status = 0, counters = 0, tmpk = 0, tmpv = 0;
  size_t ss = 0;  // sample sort region
  size_t ss_bytes = 0;
  size_t total = 0;
};

// Scratch bytes of the sample sort (samplesort_host.cpp).
size_t samplesort_ws_bytes(uint64_t n, int key_bytes, int with_payload);

inline Layout plan_layout(uint64_t n, int key_bytes, int with_payload, bool need_ss) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  const uint64_t tile = (uint64_t)os_tile(key_bytes, with_payload != 0);
  const uint64_t tiles = ceil_div(n ? n : 1, tile);
  L.df = take(sizeof(DevFeatures));
  // the digit counts start 256 bytes after the feature vector (take aligns
  // to 256), so the AUTO step reads both back with one copy
  L.dcounts = take(4 * 8 * 256);
  L.mm = take(sizeof(MinMaxPartial) * (size_t)minmax_blocks(n));
  L.hpart = take(sizeof(double) * 2048);  // one partial per reduce block (<= 65,536 / 32)
  const size_t small_parts = (size_t)hist_small_blocks(n) * HIST_SMALL_MAX_BINS;
  const size_t large_parts = (size_t)hist_large_blocks(n) * HIST_LARGE_WORDS;
  L.hist_parts = take(4 * std::max(small_parts, large_parts));
  L.corr = take(4 * 65536);
  L.hist = take(4 * 65536);
  L.offs = take(4 * 65537);
  const size_t dblocks = (size_t)std::max(digit_hist_blocks(n), hist_large_blocks(n));
  L.dparts = take(4 * dblocks * 8 * 256);
  L.doffs = take(4 * 8 * 256);
  L.status = take(8 * tiles * 256);
  L.counters = take(4 * 64);
  L.tmpk = take((size_t)key_bytes * n);
  L.tmpv = take(with_payload ? 4 * (size_t)n : 0);
  if (need_ss) {
    L.ss_bytes = samplesort_ws_bytes(n, key_bytes, with_payload);
    L.ss = take(L.ss_bytes);
  }
  L.total = o;
  return L;
}

template <typename T>
inline T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// A launch bracketed by the context's event timer.
struct ProfScope {
  ahs_context* c;
  hipStream_t s;
  ProfScope(ahs_context* c_, const char* name, hipStream_t s_, double bytes = 0.0) : c(c_), s(s_) {
    c->prof_begin(name, s, bytes);
  }
  ~ProfScope() { c->prof_end(s); }
};

// Strategy drivers (defined in sort_host.cpp / samplesort_host.cpp).
struct SortJob {
  ahs_context* ctx;
  int kk;
  int key_bytes;
  const void* kin;
  void* kout;
  const uint32_t* vin;
  uint32_t* vout;
  uint64_t n;
  void* ws;
  Layout L;
  hipStream_t s;
  DevFeatures f;   // min/max/span known
};
ahs_status run_samplesort(SortJob& j);

}  // namespace ahs
