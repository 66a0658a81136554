// ahs_features / ahs_sort: the launch sequences of the feature pass and of
// each strategy (Sec. III, Fig. 1).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ahs.h"
#include "host_internal.hpp"
#include "kernels.hpp"
#include "static_scratch.hpp"

namespace ahs {

static int key_bytes_of(ahs_dtype d) { return (d == AHS_U32 || d == AHS_F32 || d == AHS_I32) ? 4 : 8; }

// Smallest input whose AUTO min/max pass also counts the exact histogram
// (its grid then has at least 256 workgroups).
constexpr uint64_t FUSED_HIST_MIN_N = 1ull << 27;

// Radix digit counts read back to the host (up to 8 digits of 256 bins).
// A fixed array: the sort path makes no heap allocation.
struct DigitCounts {
  int ndig = 0;
  uint32_t c[8 * 256];
};

static bool partial_overlap(const void* a, const void* b, size_t bytes) {
  if (a == b || bytes == 0) return false;
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + bytes && y < x + bytes;
}


// Enqueues min/max, reads the feature header back (one sync).
static ahs_status step_minmax(SortJob& j) {
  DevFeatures* df = at<DevFeatures>(j.ws, j.L.df);
  {
    ProfScope p(j.ctx, "minmax", j.s, (double)j.key_bytes * j.n);
    AHS_HIP(j, launch_minmax(j.kk, j.kin, j.n, at<MinMaxPartial>(j.ws, j.L.mm), minmax_blocks(j.n), df, j.s),
            "minmax launch");
  }
  AHS_HIP(j, hipMemcpyAsync(j.ctx->pinned, df, sizeof(DevFeatures), hipMemcpyDeviceToHost, j.s), "copy features");
  AHS_HIP(j, hipStreamSynchronize(j.s), "synchronize");
  memcpy(&j.f, j.ctx->pinned, sizeof(DevFeatures));
  return AHS_OK;
}

// Enqueues the binned histogram of (key - min) >> shift into hist_out and
// the entropy into the device feature vector; optionally fuses ndig digit
// counts (radix upfront histogram) into the same read.
static ahs_status step_hist(SortJob& j, uint32_t* hist_out, int ndig_fused) {
  const uint32_t nbins = j.f.nbins;
  const bool large = nbins > (uint32_t)HIST_SMALL_MAX_BINS || ndig_fused > 0;
  uint32_t* parts = at<uint32_t>(j.ws, j.L.hist_parts);
  uint32_t* corr = at<uint32_t>(j.ws, j.L.corr);
  int groups;
  if (large) {
    groups = hist_large_blocks(j.n);
    AHS_HIP(j, launch_fill_u32(corr, 65536, 0u, j.s), "fill");
    ProfScope p(j.ctx, "feature_hist", j.s, (double)j.key_bytes * j.n);
    AHS_HIP(j, launch_hist_large(j.kk, j.kin, j.n, j.f.min_key, j.f.shift, parts, corr, groups, ndig_fused,
                                 at<uint32_t>(j.ws, j.L.dparts), j.s),
            "histogram launch");
  } else {
    groups = hist_small_blocks(j.n);
    ProfScope p(j.ctx, "feature_hist", j.s, (double)j.key_bytes * j.n);
    AHS_HIP(j, launch_hist_small(j.kk, j.kin, j.n, j.f.min_key, j.f.shift, nbins, parts, groups, j.s),
            "histogram launch");
  }
  int nparts = 0;
  {
    ProfScope p(j.ctx, "hist_reduce", j.s, 4.0 * nbins);
    AHS_HIP(j, launch_hist_reduce(parts, groups, nbins, large ? 1 : 0, corr, hist_out, j.n,
                                  at<double>(j.ws, j.L.hpart), &nparts, j.s),
            "histogram reduce");
    AHS_HIP(j, launch_entropy_final(at<double>(j.ws, j.L.hpart), nparts, at<DevFeatures>(j.ws, j.L.df), j.s),
            "entropy");
  }
  if (ndig_fused > 0) {
    ProfScope p(j.ctx, "digit_reduce", j.s);
    AHS_HIP(j, launch_digit_reduce(at<uint32_t>(j.ws, j.L.dparts), nullptr, groups, ndig_fused,
                                   at<uint32_t>(j.ws, j.L.dcounts), at<uint32_t>(j.ws, j.L.doffs), j.s),
            "digit reduce");
  }
  return AHS_OK;
}

// AUTO feature step with one host round trip: min/max, then both histogram
// kernels (the device plan keeps the one the span needs and skips the rest),
// the reduce with the entropy, the fused digit counts; then one read of the
// feature vector and the digit counts.  Returns the plan word.
static ahs_status step_features_auto(SortJob& j, const ahs_config& c, bool model, bool want_hist,
                                     DigitCounts* dcounts, uint32_t* plan_out) {
  DevFeatures* df = at<DevFeatures>(j.ws, j.L.df);
  uint32_t* corr = at<uint32_t>(j.ws, j.L.corr);
  FeaturePlanCfg pc = {};
  pc.enabled = 1;
  pc.kcount_minus1 = c.k_count - 1;
  pc.k_radix = c.k_radix;
  pc.n_small = c.n_small;
  pc.model = model ? 1u : 0u;
  pc.want_hist = want_hist ? 1u : 0u;
  uint32_t* parts = at<uint32_t>(j.ws, j.L.hist_parts);
  {
    // from FUSED_HIST_MIN_N keys on, the exact histogram is counted
    // speculatively in the same read (modulo counts in the histogram
    // partials), used when the span turns out small.  Below it the min/max
    // grid is too small to carry the LDS counting at full speed, and the
    // second read costs less than the counting would.
    ProfScope p(j.ctx, "minmax", j.s, (double)j.key_bytes * j.n);
    AHS_HIP(j,
            launch_minmax(j.kk, j.kin, j.n, at<MinMaxPartial>(j.ws, j.L.mm), minmax_blocks(j.n), df, j.s, &pc,
                          j.n >= FUSED_HIST_MIN_N ? parts : nullptr, corr),
            "minmax launch");
  }
  // one histogram launch: the planned large kernel counts the small exact
  // histogram too (one row per workgroup), or nothing; the min/max final
  // kernel zeroed the correction words if the packed histogram follows
  const int gl = hist_large_blocks(j.n);
  {
    ProfScope p(j.ctx, "feature_hist", j.s, (double)j.key_bytes * j.n);
    AHS_HIP(j, launch_hist_large(j.kk, j.kin, j.n, 0, 0, parts, corr, gl, 0, at<uint32_t>(j.ws, j.L.dparts), j.s, df),
            "histogram launch");
  }
  int nparts = 0;
  {
    ProfScope p(j.ctx, "hist_reduce", j.s);
    AHS_HIP(j,
            launch_hist_reduce(parts, gl, 0, 0, corr, at<uint32_t>(j.ws, j.L.hist), j.n, at<double>(j.ws, j.L.hpart),
                               &nparts, j.s, df, gl, minmax_blocks(j.n)),
            "histogram reduce");
  }
  {
    // the digit reduce also finishes the entropy
    ProfScope p(j.ctx, "digit_reduce", j.s);
    AHS_HIP(j,
            launch_digit_reduce(at<uint32_t>(j.ws, j.L.dparts), at<uint32_t>(j.ws, j.L.hist), gl, 0,
                                at<uint32_t>(j.ws, j.L.dcounts), at<uint32_t>(j.ws, j.L.doffs), j.s, df,
                                at<double>(j.ws, j.L.hpart), nparts, df),
            "digit reduce");
  }
  // the digit counts follow the feature vector in the workspace: one copy
  static_assert(sizeof(DevFeatures) <= 256, "feature vector slot");
  char* pin = static_cast<char*>(j.ctx->pinned);
  AHS_HIP(j, hipMemcpyAsync(pin, df, 256 + 4 * 8 * 256, hipMemcpyDeviceToHost, j.s), "copy features");
  AHS_HIP(j, hipStreamSynchronize(j.s), "synchronize");
  memcpy(&j.f, pin, sizeof(DevFeatures));
  const uint32_t plan = j.f.reserved;
  j.f.reserved = 0;
  // the histogram kernels read the keys only when the plan needed a
  // histogram that the min/max pass did not already count
  if (plan & (PLAN_SKIP | PLAN_FUSED)) j.ctx->prof_set_last_bytes("feature_hist", 0.0);
  const int ndig = plan_digits(plan);
  dcounts->ndig = ndig;
  if (ndig > 0) memcpy(dcounts->c, pin + 256, 4 * 256 * (size_t)ndig);
  *plan_out = plan;
  return AHS_OK;
}

// Reads back the feature vector and, if ndig > 0, the digit counts.
static ahs_status read_features(SortJob& j, int ndig, DigitCounts* counts) {
  char* pin = static_cast<char*>(j.ctx->pinned);
  AHS_HIP(j, hipMemcpyAsync(pin, at<DevFeatures>(j.ws, j.L.df), sizeof(DevFeatures), hipMemcpyDeviceToHost, j.s),
          "copy features");
  if (ndig > 0)
    AHS_HIP(j, hipMemcpyAsync(pin + 256, at<uint32_t>(j.ws, j.L.dcounts), 4 * 256 * (size_t)ndig,
                              hipMemcpyDeviceToHost, j.s),
            "copy digit counts");
  AHS_HIP(j, hipStreamSynchronize(j.s), "synchronize");
  memcpy(&j.f, pin, sizeof(DevFeatures));
  if (ndig > 0) {
    counts->ndig = ndig;
    memcpy(counts->c, pin + 256, 4 * 256 * (size_t)ndig);
  }
  return AHS_OK;
}

static int radix_digits(uint64_t span) { return std::max(1, (bitlen64(span) + 7) / 8); }

static ahs_status copy_through(SortJob& j) {
  AHS_HIP(j, launch_copy(j.kin, j.kout, (size_t)j.key_bytes * j.n, j.s), "copy");
  if (j.vin) AHS_HIP(j, launch_copy(j.vin, j.vout, 4 * (size_t)j.n, j.s), "copy");
  return AHS_OK;
}

// LSD radix, base 256, over (key - min) (Sec. III-G, eq. (4)).  Passes whose
// digit is the same for every key are skipped: they would not move a key.
static ahs_status run_radix(SortJob& j, const DigitCounts* ready_counts) {
  const int ndig = radix_digits(j.f.span);
  DigitCounts local;
  const uint32_t* counts = local.c;
  if (ready_counts) {
    counts = ready_counts->c;
  } else {
    const int nb = digit_hist_blocks(j.n);
    {
      ProfScope p(j.ctx, "digit_hist", j.s, (double)j.key_bytes * j.n);
      AHS_HIP(j, launch_digit_hist(j.kk, j.kin, j.n, j.f.min_key, ndig, at<uint32_t>(j.ws, j.L.dparts), nb, j.s),
              "digit histogram");
    }
    AHS_HIP(j, launch_digit_reduce(at<uint32_t>(j.ws, j.L.dparts), nullptr, nb, ndig, at<uint32_t>(j.ws, j.L.dcounts),
                                   at<uint32_t>(j.ws, j.L.doffs), j.s),
            "digit reduce");
    char* pin = static_cast<char*>(j.ctx->pinned);
    AHS_HIP(j, hipMemcpyAsync(pin, at<uint32_t>(j.ws, j.L.dcounts), 4 * 256 * (size_t)ndig, hipMemcpyDeviceToHost,
                              j.s),
            "copy digit counts");
    AHS_HIP(j, hipStreamSynchronize(j.s), "synchronize");
    local.ndig = ndig;
    memcpy(local.c, pin, 4 * 256 * (size_t)ndig);
  }
  int passes[8];
  int m = 0;
  for (int p = 0; p < ndig; ++p) {
    bool trivial = false;
    for (int b = 0; b < 256; ++b)
      if (counts[(size_t)p * 256 + b] == (uint32_t)j.n) trivial = true;
    if (!trivial) passes[m++] = p;
  }
  if (m == 0) return copy_through(j);

  void* tmpk = at<void>(j.ws, j.L.tmpk);
  uint32_t* tmpv = j.vin ? at<uint32_t>(j.ws, j.L.tmpv) : nullptr;
  const void* src = j.kin;
  const uint32_t* vsrc = j.vin;
  // pass q writes to the output when (m - 1 - q) is even, else to scratch
  if (j.kin == j.kout && (m % 2) == 1) {
    AHS_HIP(j, launch_copy(j.kin, tmpk, (size_t)j.key_bytes * j.n, j.s), "copy");
    src = tmpk;
  }
  if (j.vin && j.vin == j.vout && (m % 2) == 1) {
    AHS_HIP(j, launch_copy(j.vin, tmpv, 4 * (size_t)j.n, j.s), "copy");
    vsrc = tmpv;
  }
  const uint64_t tiles = ceil_div(j.n, (uint64_t)os_tile(j.key_bytes, j.vin != nullptr));
  uint32_t* status = at<uint32_t>(j.ws, j.L.status);
  const uint64_t status_words32 = tiles * 256 * status_word_bytes(j.n) / 4;
  uint32_t* counters = at<uint32_t>(j.ws, j.L.counters);
  AHS_HIP(j, launch_fill_u32(counters, 64, 0u, j.s), "fill");
  const bool mapped = j.kk == KK_F32 || j.kk == KK_F64 || j.kk == KK_I32 || j.kk == KK_I64;
  for (int q = 0; q < m; ++q) {
    const bool to_out = ((m - 1 - q) % 2) == 0;
    void* dst = to_out ? j.kout : tmpk;
    uint32_t* vdst = j.vin ? (to_out ? j.vout : tmpv) : nullptr;
    OnesweepArgs a;
    a.src = src;
    a.dst = dst;
    a.vsrc = vsrc;
    a.vdst = vdst;
    a.n = j.n;
    a.kmin = j.f.min_key;
    a.digit_shift = 8u * (uint32_t)passes[q];
    a.map_in = (mapped && q == 0) ? 1u : 0u;
    a.unmap_out = (mapped && q == m - 1) ? 1u : 0u;
    a.digit_offsets = at<uint32_t>(j.ws, j.L.doffs) + 256 * passes[q];
    a.status = status;
    a.tile_counter = counters + q;
    AHS_HIP(j, launch_fill_u32(status, status_words32, 0u, j.s), "fill");
    {
      ProfScope p(j.ctx, "onesweep_pass", j.s, (2.0 * j.key_bytes + (j.vin ? 8.0 : 0.0)) * j.n);
      AHS_HIP(j, launch_onesweep(j.kk, j.vin != nullptr, a, j.s), "onesweep launch");
    }
    src = dst;
    vsrc = vdst;
  }
  return AHS_OK;
}

// Counting sort (Sec. III-F): exact histogram of key - min, its exclusive
// scan, then keys-only expansion; with a payload the stable placement runs
// as digit scatters over the bin index (one pass per 8 bits of span).
static ahs_status run_counting(SortJob& j, bool hist_ready) {
  if (j.f.span > 65535u) return j.ctx->fail(AHS_E_UNSUPPORTED, "counting sort needs span <= 65535");
  if (j.vin) return run_radix(j, nullptr);
  uint32_t* hist = at<uint32_t>(j.ws, j.L.hist);
  if (!hist_ready) AHS_TRY(step_hist(j, hist, 0));
  uint32_t* offs = at<uint32_t>(j.ws, j.L.offs);
  {
    ProfScope p(j.ctx, "counting_scan", j.s, 8.0 * j.f.nbins);
    AHS_HIP(j, launch_scan_bins(hist, j.f.nbins, offs, j.s), "scan");
  }
  ProfScope p(j.ctx, "counting_expand", j.s, (double)j.key_bytes * j.n);
  AHS_HIP(j, launch_expand(j.kk, offs, j.f.nbins, j.f.min_key, j.kout, j.n, j.s), "expand");
  return AHS_OK;
}

static ahs_status run_small(SortJob& j) {
  ProfScope p(j.ctx, "small_sort", j.s, (2.0 * j.key_bytes + (j.vin ? 8.0 : 0.0)) * j.n);
  AHS_HIP(j, launch_small_sort(j.kk, j.kin, j.kout, j.vin, j.vout, (uint32_t)j.n, j.s), "small sort");
  return AHS_OK;
}

}  // namespace ahs

using namespace ahs;

extern "C" size_t ahs_workspace_bytes(uint64_t n, ahs_dtype dtype, int with_payload, ahs_strategy strategy) {
  if ((int)dtype < 0 || (int)dtype > (int)AHS_I64) return 0;
  const bool ss = strategy == AHS_AUTO || strategy == AHS_QUICK;
  return plan_layout(n, key_bytes_of(dtype), with_payload ? 1 : 0, ss).total;
}

static ahs_status common_checks(ahs_context* ctx, uint64_t n, ahs_dtype dtype) {
  if (!ctx) return AHS_E_INVALID_ARG;
  if ((int)dtype < 0 || (int)dtype > (int)AHS_I64) return ctx->fail(AHS_E_INVALID_ARG, "bad dtype %d", (int)dtype);
  if (n >= (1ull << 32)) return ctx->fail(AHS_E_UNSUPPORTED, "n must be below 2^32");
  return AHS_OK;
}

extern "C" ahs_status ahs_features(ahs_context* ctx, const void* d_keys, uint64_t n, ahs_dtype dtype,
                                   uint32_t* d_hist, void* d_ws, size_t ws_bytes, void* stream,
                                   ahs_feature_vector* h_out) {
  AHS_TRY(common_checks(ctx, n, dtype));
  if (!h_out) return ctx->fail(AHS_E_INVALID_ARG, "h_out is null");
  ahs_feature_vector f = {};
  f.n = n;
  if (n == 0) {
    *h_out = f;
    return AHS_OK;
  }
  if (!d_keys || !d_ws) return ctx->fail(AHS_E_INVALID_ARG, "null device pointer");
  SortJob j;
  j.ctx = ctx;
  j.kk = (int)dtype;
  j.key_bytes = key_bytes_of(dtype);
  j.kin = d_keys;
  j.kout = nullptr;
  j.vin = nullptr;
  j.vout = nullptr;
  j.n = n;
  j.ws = d_ws;
  j.L = plan_layout(n, j.key_bytes, 0, false);
  j.s = (hipStream_t)stream;
  if (ws_bytes < j.L.total) return ctx->fail(AHS_E_WORKSPACE, "workspace %zu < %zu", ws_bytes, j.L.total);
  AHS_HIP(j, hipSetDevice(ctx->device), "set device");
  AHS_TRY(step_minmax(j));
  if (j.f.nan_count) {
    f.nan_count = j.f.nan_count;
    *h_out = f;
    return ctx->fail(AHS_E_NAN, "%llu NaN keys", (unsigned long long)j.f.nan_count);
  }
  AHS_TRY(step_hist(j, d_hist ? d_hist : at<uint32_t>(j.ws, j.L.hist), 0));
  AHS_TRY(read_features(j, 0, nullptr));
  memcpy(h_out, &j.f, sizeof f);
  return AHS_OK;
}

extern "C" ahs_status ahs_sort(ahs_context* ctx, const void* d_keys_in, void* d_keys_out, const uint32_t* d_vals_in,
                               uint32_t* d_vals_out, uint64_t n, ahs_dtype dtype, ahs_strategy requested,
                               const ahs_config* cfg, void* d_ws, size_t ws_bytes, void* stream,
                               ahs_strategy* h_chosen, ahs_feature_vector* h_feats) {
  AHS_TRY(common_checks(ctx, n, dtype));
  if ((int)requested < AHS_AUTO || (int)requested > AHS_QUICK)
    return ctx->fail(AHS_E_INVALID_ARG, "strategy %d cannot be requested", (int)requested);
  if ((d_vals_in == nullptr) != (d_vals_out == nullptr))
    return ctx->fail(AHS_E_INVALID_ARG, "payload pointers must be both null or both set");
  ahs_config c;
  if (cfg) c = *cfg; else ahs_config_init(&c, AHS_PRESET_GPU);
  if (c.k_count == 0) return ctx->fail(AHS_E_INVALID_ARG, "k_count must be positive");
  if (n == 0) {
    if (h_chosen) *h_chosen = requested == AHS_AUTO ? AHS_INSERTION : requested;
    if (h_feats) *h_feats = ahs_feature_vector{};
    return AHS_OK;
  }
  if (!d_keys_in || !d_keys_out || !d_ws) return ctx->fail(AHS_E_INVALID_ARG, "null device pointer");
  const int kb = key_bytes_of(dtype);
  if (partial_overlap(d_keys_in, d_keys_out, (size_t)kb * n) ||
      (d_vals_in && partial_overlap(d_vals_in, d_vals_out, 4 * (size_t)n)))
    return ctx->fail(AHS_E_INVALID_ARG, "input and output partially overlap");

  SortJob j;
  j.ctx = ctx;
  j.kk = (int)dtype;
  j.key_bytes = kb;
  j.kin = d_keys_in;
  j.kout = d_keys_out;
  j.vin = d_vals_in;
  j.vout = d_vals_out;
  j.n = n;
  j.ws = d_ws;
  j.s = (hipStream_t)stream;
  const bool need_ss = requested == AHS_AUTO || requested == AHS_QUICK;
  j.L = plan_layout(n, kb, d_vals_in ? 1 : 0, need_ss);
  if (ws_bytes < j.L.total) return ctx->fail(AHS_E_WORKSPACE, "workspace %zu < %zu", ws_bytes, j.L.total);
  AHS_HIP(j, hipSetDevice(ctx->device), "set device");
  memset(&j.f, 0, sizeof j.f);
  j.f.n = n;

  const bool flt = dtype == AHS_F32 || dtype == AHS_F64;
  const bool want_feats = h_feats != nullptr;
  const bool model_decides = requested == AHS_AUTO && c.use_model && n >= c.ml_min_n;
  if (model_decides && !ctx->model) return ctx->fail(AHS_E_NO_MODEL, "use_model set but no model attached");
  // The FSM's first state depends on n alone: integer keys (nothing to
  // reject as NaN) whose features the caller did not ask for go straight to
  // the small-input sort, with no feature pass and no host round trip.
  if (requested == AHS_AUTO && !flt && !want_feats && n <= (uint64_t)c.n_small && n <= (uint64_t)SMALL_SORT_MAX) {
    AHS_TRY(run_small(j));
    if (h_chosen) *h_chosen = AHS_INSERTION;
    return AHS_OK;
  }
  const bool need_minmax = flt || requested != AHS_QUICK || want_feats;
  uint32_t plan = 0;
  DigitCounts dcounts;
  if (requested == AHS_AUTO) {
    AHS_TRY(step_features_auto(j, c, model_decides, want_feats, &dcounts, &plan));
  } else if (need_minmax) {
    AHS_TRY(step_minmax(j));
  }
  if (need_minmax || requested == AHS_AUTO) {
    if (j.f.nan_count) {
      if (h_feats) {
        *h_feats = ahs_feature_vector{};
        h_feats->n = n;
        h_feats->nan_count = j.f.nan_count;
      }
      return ctx->fail(AHS_E_NAN, "%llu NaN keys", (unsigned long long)j.f.nan_count);
    }
  }
  if (requested == AHS_COUNTING && (j.f.span >= c.k_count_cap || j.f.span > 65535u))
    return ctx->fail(AHS_E_UNSUPPORTED, "counting sort refused: span %llu", (unsigned long long)j.f.span);

  // Decide.  The entropy only matters for the radix test (k > k_radix), for
  // the model, or when the caller asks for the features.
  ahs_strategy s = requested;
  bool hist_ready = false;
  bool have_dcounts = false;
  if (requested == AHS_AUTO) {
    // the plan fused digit counts into the feature histogram whenever radix
    // can be the outcome (the FSM's radix test, or any span the model may
    // send to radix) and skipped the histogram where nothing needs it
    hist_ready = (plan & PLAN_SKIP) == 0;
    have_dcounts = plan_digits(plan) > 0;
    ahs_feature_vector fv;
    memcpy(&fv, &j.f, sizeof fv);
    AHS_TRY(ahs_select(&fv, &c, ctx->model, &s));
  } else if (want_feats) {
    AHS_TRY(step_hist(j, at<uint32_t>(j.ws, j.L.hist), 0));
    AHS_TRY(read_features(j, 0, nullptr));
    hist_ready = true;
  }

  ahs_status st = AHS_OK;
  switch (s) {
    case AHS_INSERTION:
      st = n <= (uint64_t)SMALL_SORT_MAX ? run_small(j) : run_radix(j, nullptr);
      break;
    case AHS_COUNTING:
      st = (j.f.span <= 65535u) ? run_counting(j, hist_ready && j.f.exact) : run_radix(j, nullptr);
      break;
    case AHS_RADIX:
      st = run_radix(j, have_dcounts ? &dcounts : nullptr);
      break;
    case AHS_QUICK:
      st = run_samplesort(j);
      break;
    default:
      st = ctx->fail(AHS_E_INVALID_ARG, "bad strategy");
  }
  if (st != AHS_OK) return st;
  if (h_chosen) *h_chosen = s;
  if (h_feats) memcpy(h_feats, &j.f, sizeof *h_feats);
  return AHS_OK;
}

// ahs_sort with its workspace in the library's fixed per-device scratch
// array: no allocation of any kind.  The array is shared by every call on
// the device (calls that overlap on one GPU race); ahs_sort clears whatever
// it needs zeroed with its own fill kernels, so stale contents from an
// earlier call are harmless.
extern "C" ahs_status ahs_sort_static(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                                      const uint32_t* d_vals_in, uint32_t* d_vals_out, uint64_t n, ahs_dtype dtype,
                                      ahs_strategy requested, const ahs_config* cfg, void* stream,
                                      ahs_strategy* h_chosen, ahs_feature_vector* h_feats) {
  using namespace ahs;
  AHS_TRY(common_checks(ctx, n, dtype));
  if ((int)requested < AHS_AUTO || (int)requested > AHS_QUICK)
    return ctx->fail(AHS_E_INVALID_ARG, "strategy %d cannot be requested", (int)requested);
  if (!ctx->static_scratch) return ctx->fail(AHS_E_DEVICE, "no static scratch on device %d", ctx->device);
  const size_t need = ahs_workspace_bytes(n, dtype, d_vals_in != nullptr ? 1 : 0, requested);
  if (need > STATIC_SCRATCH_BYTES)
    return ctx->fail(AHS_E_WORKSPACE, "%llu keys need %zu bytes of scratch; the static scratch holds %zu",
                     (unsigned long long)n, need, STATIC_SCRATCH_BYTES);
  return ahs_sort(ctx, d_keys_in, d_keys_out, d_vals_in, d_vals_out, n, dtype, requested, cfg, ctx->static_scratch,
                  STATIC_SCRATCH_BYTES, stream, h_chosen, h_feats);
}
