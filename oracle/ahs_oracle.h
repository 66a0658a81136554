/*
 * Adaptive Hybrid Sort -- CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded C
 * implementation of what the GPU library computes, written from the paper
 * (Adaptive Hybrid Sort, arXiv 2506.20677).  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load or run it; the product
 * library never links, loads or calls it, and it shares no code, header,
 * table or helper with the product.
 *
 * Paper passages followed (section / equation / listing / table):
 *   - state vector v = (n, k, H), k = max - min + 1, H = -sum p log2 p:
 *     Sec. III-A (Algorithm Design); Sec. III-H.
 *   - decision FSM (n <= 20 insertion; k <= K_c counting; k > 1e6 and
 *     H < 0.7 log2 k radix; else quicksort): Sec. III intro, Sec. III-A,
 *     Fig. 2, Listing 6; thresholds Table II.
 *   - insertion sort: Sec. III-E, Listing 1.
 *   - counting sort (count, prefix, backward placement): Sec. III-F,
 *     Listing 2.
 *   - radix sort, base 256 for large ranges, d = ceil(log_256 k) digits:
 *     Sec. III-G, eq. (4) (Lemma 3.1).
 *   - quicksort with a median-of-three pivot: Sec. III-G.1, Listing 4.
 *   - optional learned strategy predictor over (n, k, H), used for n >= 1000
 *     with static rules below: Sec. III-H, Listing 5, Table IV.
 *   - empty input exits at once; all-equal input (k = 1) needs no sorting:
 *     Sec. III-K.
 *
 * Readings where the paper is silent, garbled or self-contradictory (each
 * also listed in the design notes of the repository):
 *   R1  K_c is a configuration value (preset 4096; paper presets 1000, 1024;
 *       preset 3 holds n_small 48 and K_c 5000, recalibrated by eq. (1)).
 *   R2  The entropy test is relative: H < h_ratio * log2(B), strict.
 *   R3  H is computed over at most 65,536 bins of (m - min) >> s with the
 *       smallest such shift s; exact per value when span <= 65,535.  The
 *       radix test compares against log2(B), B = number of bins.
 *   R5  Radix is always base 256 over (m - min), d = max(1, ceil(bitlen(span)/8)).
 *   R7  Listing 4 drops duplicates of the pivot; the oracle partitions three
 *       ways (<, ==, >), keeping input order inside each part.
 *   R8  Every sort is stable, so payloads are defined uniquely.
 *   R10 k = span + 1 can be 2^64, so span is stored; k <= K_c <=> span <= K_c-1,
 *       k > k_radix <=> span >= k_radix.
 *   R11 Floating keys are ordered through a sign-flip bit map (-0.0 < +0.0,
 *       NaN rejected); the paper itself rejects non-integers (Sec. III-K).
 *
 * All functions return REF_OK (0) or a negative REF_E_* code.
 */
#ifndef AHS_ORACLE_H
#define AHS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { REF_U32 = 0, REF_U64 = 1, REF_F32 = 2, REF_F64 = 3, REF_I32 = 4, REF_I64 = 5 };

enum {
  REF_AUTO = 0,
  REF_COUNTING = 1,
  REF_RADIX = 2,
  REF_QUICK = 3,
  REF_INSERTION = 4
};

enum {
  REF_OK = 0,
  REF_E_INVALID_ARG = -1,
  REF_E_UNSUPPORTED = -2,
  REF_E_NAN = -3,
  REF_E_OOM = -5,
  REF_E_NO_MODEL = -7,
  REF_E_DEPTH = -8,
  REF_E_PARSE = -9
};

/* Feature vector (Sec. III-A).  min/max are in the mapped ordered-unsigned
 * key space, zero-extended to 64 bits. */
typedef struct {
  uint64_t n;
  uint64_t min_key;
  uint64_t max_key;
  uint64_t span;        /* max - min; k = span + 1 */
  uint64_t nan_count;
  uint32_t shift;       /* bin = (m - min) >> shift */
  uint32_t nbins;       /* B = (span >> shift) + 1, at most 65,536 */
  uint32_t exact;       /* 1 iff shift == 0 (one bin per value) */
  uint32_t reserved;
  double entropy_bits;  /* H = -sum_{c>0} (c/n) log2(c/n), FP64 */
  double entropy_ratio; /* H / log2(B), 0 when B == 1 */
} ref_features;

/* Decision thresholds (Sec. III-A, Table II). */
typedef struct {
  uint32_t n_small;     /* INSERTION when n <= n_small */
  uint32_t use_model;   /* consult the learned predictor when n >= ml_min_n */
  uint64_t k_count;     /* COUNTING when k <= k_count */
  uint64_t k_radix;     /* RADIX requires k > k_radix ... */
  double h_ratio;       /* ... and H < h_ratio * log2(B) */
  uint64_t ml_min_n;
  uint64_t k_count_cap; /* COUNTING refused when span >= k_count_cap */
} ref_config;

typedef struct ref_model ref_model;

/* Presets: 0 = GPU default (K_c 4096), 1 = paper text (K_c 1000),
 * 2 = paper Table II (K_c 1024). */
int ref_config_init(ref_config* cfg, int preset);

/* Order-preserving key map to 64-bit unsigned (Sec. III-K; reading R11). */
int ref_map_keys(int dtype, const void* keys, uint64_t n, uint64_t* mapped,
                 uint64_t* nan_count);
int ref_unmap_keys(int dtype, const uint64_t* mapped, uint64_t n, void* keys);

/* Features (Sec. III-A).  hist, if non-null, receives exactly nbins counts.
 * Returns REF_E_NAN (with n and nan_count filled) when a NaN is present. */
int ref_features_compute(int dtype, const void* keys, uint64_t n,
                         uint32_t* hist, ref_features* out);

/* Strategy selection (Sec. III-A FSM; Sec. III-H predictor). */
int ref_select(const ref_features* f, const ref_config* cfg,
               const ref_model* model, int* strategy);

/* Full method: features, decision, the chosen (or forced) sort.  vals_in and
 * vals_out are both null or both non-null.  Forced REF_INSERTION is allowed
 * here so that the four sorts can be compared with each other. */
int ref_sort(int dtype, const void* keys_in, void* keys_out,
             const uint32_t* vals_in, uint32_t* vals_out, uint64_t n,
             int requested, const ref_config* cfg, const ref_model* model,
             int* chosen, ref_features* feats);

/* Learned predictor in the project's own text format (Sec. III-H). */
int ref_model_load(const char* path, ref_model** out);
void ref_model_free(ref_model* m);
int ref_model_predict(const ref_model* m, const ref_features* f, int* strategy);

#ifdef __cplusplus
}
#endif
#endif
