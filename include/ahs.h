/*
 * ahs.h -- C ABI of the MI355X (gfx950) Adaptive Hybrid Sort library.
 *
 * Adaptive Hybrid Sort (arXiv 2506.20677) computes a state vector
 * v = (n, k, H) over its input -- size, value range k = max - min + 1 and the
 * Shannon entropy H = -sum p_i log2 p_i of the value distribution (Sec. III-A)
 * -- and a decision engine (a finite-state machine, Sec. III-A and Fig. 2,
 * optionally a learned predictor, Sec. III-H) dispatches to insertion sort
 * (n <= 20), counting sort (small k), radix sort (k > 1e6 with low entropy)
 * or quicksort (everything else).  The calls below follow that statement of
 * the problem: ahs_features computes v, ahs_select runs the decision engine,
 * ahs_sort runs the whole method (or one forced strategy) on device buffers.
 *
 * Conventions shared by every call:
 *   - Every call returns an ahs_status.  On error no caller buffer has been
 *     written, and ahs_last_error() holds a message.
 *   - Device pointers ("d_") are HIP device memory owned by the caller.  The
 *     library keeps no pointer after a call returns.  Host pointers ("h_")
 *     are ordinary host memory.
 *   - Keys are contiguous arrays of n elements of the given dtype.  Floating
 *     keys are ordered by an order-preserving bit map (sign bit set: flip all
 *     bits; clear: set the sign bit), so -0.0 sorts before +0.0, -inf first
 *     and +inf last; NaN is rejected with AHS_E_NAN.  The paper accepts only
 *     integers (Sec. III-K); floats are this library's extension.  Signed
 *     integer keys (AHS_I32, AHS_I64) are ordered by their value through a
 *     flip of the sign bit.
 *   - Payloads are optional uint32 arrays permuted with the keys.  Every
 *     strategy is stable, so the payload result is unique.
 *   - `stream` is a hipStream_t passed as void* (0 = the null stream).  Calls
 *     that must decide on the host (AUTO, float NaN checks, radix pass
 *     planning) synchronise that stream once or twice; the others only
 *     enqueue work.  AUTO on integer keys with n <= n_small and no feature
 *     request only enqueues: that state depends on n alone.
 *   - `d_ws` is caller-provided device scratch of at least
 *     ahs_workspace_bytes(...) bytes, 256-byte aligned.  The library never
 *     allocates device memory inside a sort call.
 *   - One context per host thread; contexts are not thread-safe.
 *   - n must be below 2^32.
 */
#ifndef AHS_H
#define AHS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key types.  Floating keys are ordered by their IEEE bit pattern mapped
 * order-preservingly onto unsigned integers (-0.0 before +0.0, infinities at
 * the ends, NaN refused by the single-array calls); signed keys by flipping
 * the sign bit, the GPU counterpart of the two-bucket signed radix of
 * Listing 7.  Features (min_key, max_key) are reported in the mapped domain. */
typedef enum { AHS_U32 = 0, AHS_U64 = 1, AHS_F32 = 2, AHS_F64 = 3, AHS_I32 = 4, AHS_I64 = 5 } ahs_dtype;

/* AHS_INSERTION is only reported: it is the n <= n_small state of the FSM
 * (Sec. III-A, Listing 1); it cannot be requested. */
typedef enum {
  AHS_AUTO = 0,
  AHS_COUNTING = 1,
  AHS_RADIX = 2,
  AHS_QUICK = 3,
  AHS_INSERTION = 4
} ahs_strategy;

typedef enum {
  AHS_OK = 0,
  AHS_E_INVALID_ARG = -1, /* bad pointer, size, dtype, strategy or overlap */
  AHS_E_UNSUPPORTED = -2, /* n >= 2^32, or forced COUNTING with span >= k_count_cap */
  AHS_E_NAN = -3,         /* a floating key is NaN */
  AHS_E_WORKSPACE = -4,   /* ws_bytes below the required size */
  AHS_E_OOM = -5,         /* host allocation failed (context creation only) */
  AHS_E_DEVICE = -6,      /* a HIP runtime call failed */
  AHS_E_NO_MODEL = -7,    /* use_model set but no model attached */
  AHS_E_PARSE = -9        /* model file malformed */
} ahs_status;

/* The state vector v = (n, k, H) of Sec. III-A, plus what the GPU needs.
 * min_key/max_key are in the mapped ordered-unsigned space, zero-extended to
 * 64 bits.  k = span + 1 is not stored (it can be 2^64).  The entropy is
 * taken over nbins = (span >> shift) + 1 <= 65,536 bins of
 * (key - min) >> shift, shift the smallest such value; exact == 1 means one
 * bin per value.  entropy_ratio = H / log2(nbins), 0 when nbins == 1. */
typedef struct {
  uint64_t n;
  uint64_t min_key;
  uint64_t max_key;
  uint64_t span;
  uint64_t nan_count;
  uint32_t shift;
  uint32_t nbins;
  uint32_t exact;
  uint32_t reserved;
  double entropy_bits;
  double entropy_ratio;
} ahs_feature_vector;

/* Decision thresholds (Sec. III-A; Table II; Sec. III-H).
 *   INSERTION  if n <= n_small
 *   COUNTING   else if k <= k_count            (span <= k_count - 1)
 *   RADIX      else if k > k_radix and H < h_ratio * log2(nbins)
 *   QUICK      otherwise
 * With use_model and n >= ml_min_n the attached model decides instead,
 * except that a COUNTING prediction with span >= k_count_cap falls back to
 * the FSM.  Forced COUNTING is refused when span >= k_count_cap. */
typedef struct {
  uint32_t n_small;
  uint32_t use_model;
  uint64_t k_count;
  uint64_t k_radix;
  double h_ratio;
  uint64_t ml_min_n;
  uint64_t k_count_cap;
} ahs_config;

enum {
  AHS_PRESET_GPU = 0,              /* k_count 4096 (default) */
  AHS_PRESET_PAPER_TEXT = 1,       /* k_count 1000 (Sec. III-A) */
  AHS_PRESET_PAPER_TABLE2 = 2,     /* k_count 1024 (Table II) */
  AHS_PRESET_MI355X_CALIBRATED = 3 /* n_small 48, k_count 5000: eq. (1) of Sec. III-C (alpha 0.7) minimised
                                      over n_t in [10, 50], k_t in [500, 5000] on MI355X timings */
};

typedef struct ahs_context ahs_context;
typedef struct ahs_model ahs_model;

/* Fills *cfg with a preset: n_small 20 (48 for the calibrated preset),
 * k_radix 1e6, h_ratio 0.7, ml_min_n 1000, k_count_cap 65,536, use_model 0,
 * and the preset's k_count.  An unknown preset is AHS_E_INVALID_ARG. */
ahs_status ahs_config_init(ahs_config* cfg, int preset);

/* Creates host-side state bound to HIP device `device`: device properties,
 * a small pinned staging buffer, per-kernel timing, the optional model, and
 * the device address of the library's fixed ahs_sort_static scratch on that
 * device (looked up once per device; the HIP runtime places the array when
 * it loads the library's code there).  No other device memory is
 * allocated. */
ahs_status ahs_context_create(int device, ahs_context** out);
void ahs_context_destroy(ahs_context* ctx);

/* Attaches (borrows) a model used when cfg->use_model is set; NULL detaches. */
ahs_status ahs_context_set_model(ahs_context* ctx, const ahs_model* model);

/* Number of compute units of the context's device. */
uint32_t ahs_device_cu_count(const ahs_context* ctx);

/* Bytes of scratch that ahs_features (strategy ignored) or ahs_sort with
 * `strategy` needs for n keys of `dtype`; AUTO returns the maximum over the
 * strategies.  Depends only on the arguments, not on the data. */
size_t ahs_workspace_bytes(uint64_t n, ahs_dtype dtype, int with_payload, ahs_strategy strategy);

/* Features (Sec. III-A): n, min, max, span, shift, nbins, the binned
 * entropy and its ratio, and the NaN count.  If d_hist is non-null it
 * receives the nbins counts (capacity: 65,536 uint32).  Blocks until *h_out
 * is valid.  NaN keys: returns AHS_E_NAN with n and nan_count set. */
ahs_status ahs_features(ahs_context* ctx, const void* d_keys, uint64_t n, ahs_dtype dtype,
                        uint32_t* d_hist, void* d_ws, size_t ws_bytes, void* stream,
                        ahs_feature_vector* h_out);

/* Decision engine (Sec. III-A FSM; Sec. III-H predictor).  Pure host
 * function; `model` may be NULL unless cfg->use_model is set and
 * f->n >= cfg->ml_min_n (then AHS_E_NO_MODEL). */
ahs_status ahs_select(const ahs_feature_vector* f, const ahs_config* cfg, const ahs_model* model,
                      ahs_strategy* out);

/* The whole method (Sec. III, Fig. 1): features, decision, then the chosen
 * sort -- or the requested strategy when it is not AHS_AUTO.  Sorts n keys
 * ascending and stably into d_keys_out; d_vals_in/d_vals_out are both NULL
 * or both non-NULL and are permuted alike.  In-place (in == out) is allowed;
 * partial overlap is AHS_E_INVALID_ARG.  cfg NULL means AHS_PRESET_GPU.
 * h_chosen (nullable) receives the strategy that ran (AHS_INSERTION for
 * n <= n_small under AUTO).  h_feats (nullable) receives the full feature
 * vector; asking for it makes the call compute the entropy even when the
 * decision does not need it.  n == 0 returns AHS_OK without launching. */
ahs_status ahs_sort(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                    const uint32_t* d_vals_in, uint32_t* d_vals_out, uint64_t n, ahs_dtype dtype,
                    ahs_strategy requested, const ahs_config* cfg, void* d_ws, size_t ws_bytes,
                    void* stream, ahs_strategy* h_chosen, ahs_feature_vector* h_feats);

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): ahs_sort
 * with no workspace argument.  Its scratch is a fixed array of
 * AHS_STATIC_SCRATCH_BYTES inside the library, one per GPU, allocated when
 * the library's code is loaded on that GPU and held until the process ends;
 * its device address is looked up once per device by ahs_context_create.
 * The call allocates nothing (no hipMalloc, hipFree or host heap).  Inputs,
 * outputs and every other argument behave as in ahs_sort.  A call whose
 * ahs_workspace_bytes(n, dtype, with_payload, requested) exceeds
 * AHS_STATIC_SCRATCH_BYTES returns AHS_E_WORKSPACE before any launch (about
 * 4.2e6 u32 keys under AUTO, 2.1e6 u64 keys with payload).  All calls on
 * one GPU share its array, and it keeps the last call's contents: calls that
 * overlap in time on one GPU (other streams or host threads) race and give
 * undefined results; serialise them. */
#define AHS_STATIC_SCRATCH_BYTES (64ull << 20)
ahs_status ahs_sort_static(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                           const uint32_t* d_vals_in, uint32_t* d_vals_out, uint64_t n, ahs_dtype dtype,
                           ahs_strategy requested, const ahs_config* cfg, void* stream,
                           ahs_strategy* h_chosen, ahs_feature_vector* h_feats);

/* Batched segmented sort: nseg independent arrays stored back to back,
 * segment s occupying [d_offsets[s], d_offsets[s+1]) of the key (and
 * payload) arrays; d_offsets is a device array of nseg + 1 non-decreasing
 * uint64 with d_offsets[nseg] == n_total.  Each segment's output equals
 * ahs_sort on that segment alone (stable ascending order), and its decision
 * is the FSM of Sec. III-A on its own features (the entropy test uses the
 * device's FP64 log2, so a decision may differ from ahs_select only where
 * H lies within rounding of h_ratio * log2(nbins)).  Segments of at most
 * 8,192 keys are queued by size class (up to 1,024 / 2,048 / 4,096 / 8,192
 * keys) and each class is sorted wholly in LDS by one fused kernel that also
 * computes the segment's features and decision.  Larger segments get their
 * min/max and, where the span reaches k_radix, their entropy before they
 * are sorted, and their decision picks the kernels that sort them, all such
 * segments together: COUNTING and RADIX segments go through segmented
 * stable LSD passes over the 8-bit digits of key - min that vary (Sec.
 * III-F, III-G; a counting sort over at most 2^16 values is the same stable
 * scatter by the bin index), QUICK segments and segments holding NaN keys
 * through the sample-sort levels (Sec. III-G.1).  A forced strategy picks
 * the family the same way.  When d_feats is requested the large segments'
 * feature vectors are taken from their sorted output (features do not
 * depend on key order).
 * d_chosen (nullable, nseg bytes) receives each segment's strategy code
 * (AHS_* values; 0xFD marks a segment holding NaN keys, whose output is its
 * keys ordered by the bit map, NaNs at the ends).  d_feats (nullable, nseg
 * entries) receives each segment's feature vector.  cfg->use_model is not
 * supported here (AHS_E_UNSUPPORTED).  A forced strategy is reported for
 * every segment.  In-place (in == out) is allowed.  n_total may exceed
 * 2^32; each segment must hold fewer than 2^32 keys.  Workspace:
 * ahs_segmented_workspace_bytes(n_total, nseg, dtype, with_payload).
 *
 * ahs_sort_segmented blocks: it reads the classification back once (invalid
 * offsets give AHS_E_INVALID_ARG before any output is written) and once per
 * sample-sort level (2-3 reads for segments up to 2^20 keys). */
size_t ahs_segmented_workspace_bytes(uint64_t n_total, uint32_t nseg, ahs_dtype dtype, int with_payload);
ahs_status ahs_sort_segmented(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                              const uint32_t* d_vals_in, uint32_t* d_vals_out, const uint64_t* d_offsets,
                              uint32_t nseg, uint64_t n_total, ahs_dtype dtype, ahs_strategy requested,
                              const ahs_config* cfg, void* d_ws, size_t ws_bytes, void* stream,
                              uint8_t* d_chosen, ahs_feature_vector* d_feats);

/* Enqueue-only form of ahs_sort_segmented: never synchronises, so it can be
 * captured in a hipGraph.  Every kernel reads its work count from the
 * device; the sample sort launches enough levels for segments of at most
 * max_seg_hint keys (0: n_total) to shrink 64-fold per level, plus one.
 * Errors found on the device are reported in *d_status (a device uint32,
 * required), written by the last kernel: 0 success; bit 0 invalid offsets
 * (nothing else was written); bit 1 sample-sort table overflow; bit 2 a
 * segment larger than max_seg_hint remained unsplit (its output is not
 * sorted); bit 3 a segment holds more than max_seg_hint keys (the level
 * count and look-back word width were sized for the hint, so its output
 * may be wrong).  Host-side argument errors return a status as usual. */
ahs_status ahs_sort_segmented_async(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                                    const uint32_t* d_vals_in, uint32_t* d_vals_out, const uint64_t* d_offsets,
                                    uint32_t nseg, uint64_t n_total, uint64_t max_seg_hint, ahs_dtype dtype,
                                    ahs_strategy requested, const ahs_config* cfg, void* d_ws, size_t ws_bytes,
                                    void* stream, uint8_t* d_chosen, ahs_feature_vector* d_feats,
                                    uint32_t* d_status);

/* hipGraph of one ahs_sort_segmented_async call with these exact pointers
 * and sizes (captured on a private stream; the library's event timer is
 * off while capturing).  ahs_graph_launch replays it on `stream`; the
 * buffers must stay allocated while the graph lives.  Replays sort whatever
 * the input buffers hold at replay time. */
typedef struct ahs_graph ahs_graph;
ahs_status ahs_sort_segmented_capture(ahs_context* ctx, const void* d_keys_in, void* d_keys_out,
                                      const uint32_t* d_vals_in, uint32_t* d_vals_out, const uint64_t* d_offsets,
                                      uint32_t nseg, uint64_t n_total, uint64_t max_seg_hint, ahs_dtype dtype,
                                      ahs_strategy requested, const ahs_config* cfg, void* d_ws, size_t ws_bytes,
                                      uint8_t* d_chosen, ahs_feature_vector* d_feats, uint32_t* d_status,
                                      ahs_graph** out);
ahs_status ahs_graph_launch(ahs_graph* graph, void* stream);
void ahs_graph_destroy(ahs_graph* graph);

/* Size-class kernel variants of the batched sort.  h_caps[4] holds, for the
 * classes up to 1,024 / 2,048 / 4,096 / 8,192 keys, the LDS capacity of the
 * kernel variant that sorts it (1,024 / 2,048 / 4,096 with 256 threads, or
 * 8,192 with 512 threads; a class's variant must cover it).  Every variant
 * gives identical results; only speed differs.  ahs_segmented_autotune
 * times every admissible variant per class on synthetic segments (about
 * 2^22 keys per class, allocated and freed inside the call), keeps the
 * fastest in the context for (dtype, with_payload) and reports the choice
 * (h_caps, nullable) and its kernel time in ms (h_ms[4], nullable).  It
 * synchronises the stream. */
ahs_status ahs_segmented_autotune(ahs_context* ctx, ahs_dtype dtype, int with_payload, void* stream, int* h_caps,
                                  double* h_ms);
/* Tile of the segmented LSD radix passes that sort the large COUNTING and
 * RADIX segments of a batch (Sec. III-F, III-G), in keys per tile: 512
 * threads times the items per thread of one of two shapes per key size and
 * payload flag (u32: 8,192 or 12,288; u32 with payload and u64: 6,144 or
 * 9,216; u64 with payload: 4,096 or 6,144).  ahs_segmented_autotune also
 * times both on a synthetic batch of large segments sorted with RADIX
 * forced and keeps the faster.  Results do not depend on the choice.
 * Setting a size that is not one of the two is AHS_E_INVALID_ARG. */
ahs_status ahs_segmented_get_radix_tile(ahs_context* ctx, ahs_dtype dtype, int with_payload, uint32_t* h_keys_per_tile);
ahs_status ahs_segmented_set_radix_tile(ahs_context* ctx, ahs_dtype dtype, int with_payload, uint32_t keys_per_tile);
ahs_status ahs_segmented_get_variants(ahs_context* ctx, ahs_dtype dtype, int with_payload, int* h_caps);
ahs_status ahs_segmented_set_variants(ahs_context* ctx, ahs_dtype dtype, int with_payload, const int* h_caps);

/* Serving loop.  Sort requests of different sizes and key types arrive
 * over time; the server keeps their buffers on the device inside one arena
 * of hbm_budget_bytes (allocated by ahs_server_create), admits a batch only
 * when its buffers (inputs, outputs, payloads, offsets and the batched
 * sort's workspace) fit in the free part of the arena, and runs batches on
 * `slots` streams at once.  Batching is continuous: whenever a slot is
 * free, the oldest pending request and the later pending requests of the
 * same key type and payload flag (in arrival order, up to max_batch_keys
 * keys and max_batch_requests requests; the oldest is always taken) form a
 * batch, sorted by the enqueue-only batched sort.  Each request's result is
 * identical to ahs_sort(AUTO) of that request alone; its reported strategy
 * is its own FSM decision.  A request that cannot fit even in an empty arena
 * completes with AHS_E_OOM.  Latency = completion (the batch's completion
 * event, on the server clock) - arrival (given, or the submit time).
 * One host thread drives a server; the calls are not thread-safe.
 *
 * ahs_server_submit: the input (and payload) buffers are the caller's and
 * must stay unmodified until the request completes; the server records an
 * event on src_stream (the stream that produced the input) and orders its
 * copy after it.  arrival_ms < 0 means now (ahs_server_now_ms clock).
 * ahs_server_poll: advances the loop, returns up to `max` finished requests
 * (each once), waiting up to wait_ms for at least one while work remains.
 * Results point into the arena (d_keys_out, d_vals_out) and stay valid until
 * ahs_server_release(id); a batch's memory returns to the arena when all its
 * requests are released, so unreleased results hold back admission. */
typedef struct ahs_server ahs_server;
typedef struct {
  uint64_t hbm_budget_bytes;     /* arena size: the admission limit */
  uint64_t max_batch_keys;
  uint32_t max_batch_requests;   /* 1..65535 */
  uint32_t slots;                /* batches in flight at once, 1..16 */
  uint32_t autotune;             /* run ahs_segmented_autotune for every key type at creation */
  uint32_t lazy_dispatch;        /* 1: submit only queues; batches are formed and launched by poll */
  ahs_config cfg;                /* decision thresholds; use_model must be 0 */
} ahs_server_config;
typedef struct {
  uint64_t id;
  int32_t status;                /* AHS_OK, AHS_E_OOM, or AHS_E_DEVICE */
  int32_t chosen;                /* the request's strategy code (0xFD: holds NaN keys) */
  uint64_t n;
  ahs_dtype dtype;
  int32_t reserved;
  const void* d_keys_out;
  const uint32_t* d_vals_out;    /* null without payload */
  double arrival_ms, done_ms;
} ahs_server_result;
typedef struct {
  uint64_t submitted, completed, failed, pending, running_batches, batches;
  uint64_t keys_completed;
  double mean_batch_requests;
  double p50_ms, p99_ms, max_ms, mean_ms;   /* latency of completed requests (nearest rank) */
  double first_arrival_ms, last_done_ms;
  double gkeys_per_s;                        /* keys completed / (last completion - first arrival) */
  uint64_t arena_used_bytes, arena_peak_bytes;
} ahs_server_statistics;
void ahs_server_config_init(ahs_server_config* cfg);
ahs_status ahs_server_create(int device, const ahs_server_config* cfg, ahs_server** out);
double ahs_server_now_ms(ahs_server* server);
ahs_status ahs_server_submit(ahs_server* server, ahs_dtype dtype, uint64_t n, const void* d_keys,
                             const uint32_t* d_vals, void* src_stream, double arrival_ms, uint64_t* out_id);
ahs_status ahs_server_poll(ahs_server* server, ahs_server_result* out, uint32_t max, uint32_t* count,
                           double wait_ms);
ahs_status ahs_server_release(ahs_server* server, uint64_t id);
ahs_status ahs_server_stats(ahs_server* server, ahs_server_statistics* out);
void ahs_server_destroy(ahs_server* server);

/* Learned predictor (Sec. III-H, Listing 5): gradient-boosted trees over
 * (n, k, H) in the project's text format
 *   ahs-gbt 1 / num_class 3 / base_score s0 s1 s2 / num_trees T /
 *   T x { tree <class> <nodes>; nodes x { <id> split <f> <thr> <l> <r> |
 *                                          <id> leaf <value> } }
 * (features 0 = n, 1 = k, 2 = H; left when x < thr; classes 0 COUNTING,
 * 1 RADIX, 2 QUICK; largest summed score wins, ties to the lower class). */
ahs_status ahs_model_load(const char* path, ahs_model** out);
void ahs_model_free(ahs_model* m);
ahs_status ahs_model_predict(const ahs_model* m, const ahs_feature_vector* f, ahs_strategy* out);

/* Per-kernel timing with HIP events on the launch stream.  When enabled,
 * every kernel launch of the context is bracketed by two events and tagged
 * with its algorithmic HBM bytes (the reads and writes the method needs:
 * keys, payloads, histograms -- not the kernel's own scratch); totals are
 * collected (with an event synchronisation) by ahs_profile_query.  `kernel`
 * is a family name such as "onesweep_pass", "minmax", "feature_hist",
 * "ss_scatter".  Any output pointer may be NULL. */
ahs_status ahs_profile_enable(ahs_context* ctx, int on);
ahs_status ahs_profile_reset(ahs_context* ctx);
ahs_status ahs_profile_query(ahs_context* ctx, const char* kernel, uint64_t* launches,
                             double* total_ms, double* algo_bytes);
/* Writes "name launches total_ms algo_bytes\n" lines for every kernel seen;
 * returns the number of bytes needed (including the terminating zero). */
size_t ahs_profile_dump(ahs_context* ctx, char* buf, size_t len);

const char* ahs_status_str(ahs_status s);
const char* ahs_last_error(const ahs_context* ctx);

#ifdef __cplusplus
}
#endif
#endif
