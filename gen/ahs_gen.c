/*
 * Seeded synthetic input generators shared by the tests, the benchmark and
 * the smoke check.  Holds none of the sorting method's arithmetic: only
 * random draws and the composition of workloads (uniform keys, Zipf ranks,
 * Normal values, positional edits).
 *
 * Core generator: counter-based SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014).  Word i of stream
 * t under seed S is  mix64(base(S, t) + (i + 1) * GAMMA)  with
 * base(S, t) = mix64(S * GAMMA + mix64(t + GAMMA)), GAMMA the golden-ratio
 * increment and mix64 the SplitMix64 finaliser.  Any word can be computed
 * independently, so the fills below run in parallel and stay deterministic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t stream_base(uint64_t seed, uint64_t stream) {
  return mix64(seed * GAMMA + mix64(stream + GAMMA));
}

static inline uint64_t word_at(uint64_t base, uint64_t i) {
  return mix64(base + (i + 1u) * GAMMA);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double unit53(uint64_t w) { return (double)(w >> 11) * (1.0 / 9007199254740992.0); }

void gen_words(uint64_t seed, uint64_t stream, uint64_t n, uint64_t* out) {
  uint64_t b = stream_base(seed, stream);
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) out[i] = word_at(b, (uint64_t)i);
}

/* high 32 bits of each word, masked */
void gen_u32(uint64_t seed, uint64_t stream, uint64_t n, uint32_t mask, uint32_t* out) {
  uint64_t b = stream_base(seed, stream);
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) out[i] = (uint32_t)(word_at(b, (uint64_t)i) >> 32) & mask;
}

void gen_u64(uint64_t seed, uint64_t stream, uint64_t n, uint64_t mask, uint64_t* out) {
  uint64_t b = stream_base(seed, stream);
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) out[i] = word_at(b, (uint64_t)i) & mask;
}

/* uniform integers in [0, range) by multiply-shift of the high 32 bits
 * (range < 2^32), used for positions */
void gen_index(uint64_t seed, uint64_t stream, uint64_t n, uint64_t range, uint64_t* out) {
  uint64_t b = stream_base(seed, stream);
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) out[i] = ((word_at(b, (uint64_t)i) >> 32) * range) >> 32;
}

/* m distinct values in draw order; bits = 32 takes the high 32 bits of each
 * word, 64 the whole word.  Returns the number of words consumed. */
uint64_t gen_distinct(uint64_t seed, uint64_t stream, uint32_t m, int bits, uint64_t* out) {
  uint64_t b = stream_base(seed, stream), i = 0;
  uint32_t got = 0, j;
  while (got < m) {
    uint64_t w = word_at(b, i++);
    int dup = 0;
    if (bits == 32) w >>= 32;
    for (j = 0; j < got; j++)
      if (out[j] == w) { dup = 1; break; }
    if (!dup) out[got++] = w;
  }
  return i;
}

/* Zipf(s, m) rank indices in [0, m): inverse CDF by binary search over the
 * FP64 cumulative sums of r^-s, r = 1..m. */
int gen_zipf_index(uint64_t seed, uint64_t stream, uint64_t n, double s, uint32_t m, uint32_t* out) {
  double* cdf = (double*)malloc((size_t)m * sizeof(double));
  double acc = 0.0;
  uint64_t b = stream_base(seed, stream);
  uint32_t r;
  int64_t i;
  if (!cdf || m == 0) { free(cdf); return -1; }
  for (r = 0; r < m; r++) { acc += pow((double)(r + 1), -s); cdf[r] = acc; }
  for (r = 0; r < m; r++) cdf[r] /= acc;
  cdf[m - 1] = 1.0;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) {
    double u = unit53(word_at(b, (uint64_t)i));
    uint32_t lo = 0, hi = m - 1;
    while (lo < hi) {
      uint32_t mid = lo + (hi - lo) / 2;
      if (cdf[mid] > u) hi = mid; else lo = mid + 1;
    }
    out[i] = lo;
  }
  free(cdf);
  return 0;
}

/* Normal(0, sigma) by Box-Muller in FP64; element i uses words 2i, 2i+1. */
void gen_normal(uint64_t seed, uint64_t stream, uint64_t n, double sigma, double* out) {
  uint64_t b = stream_base(seed, stream);
  const double two_pi = 6.283185307179586476925286766559;
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) {
    double u1 = ((double)(word_at(b, 2u * (uint64_t)i) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    double u2 = unit53(word_at(b, 2u * (uint64_t)i + 1u));
    out[i] = sigma * sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
  }
}

/* Exponential inter-arrival gaps with the given rate. */
void gen_exponential(uint64_t seed, uint64_t stream, uint64_t n, double rate, double* out) {
  uint64_t b = stream_base(seed, stream);
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) {
    double u = ((double)(word_at(b, (uint64_t)i) >> 11) + 1.0) * (1.0 / 9007199254740992.0);
    out[i] = -log(u) / rate;
  }
}

/* Uniform doubles in [0, 1). */
void gen_unit(uint64_t seed, uint64_t stream, uint64_t n, double* out) {
  uint64_t b = stream_base(seed, stream);
  int64_t i;
#pragma omp parallel for schedule(static)
  for (i = 0; i < (int64_t)n; i++) out[i] = unit53(word_at(b, (uint64_t)i));
}

/* count sequential transpositions of positions drawn from the stream,
 * applied in order to an array of elements of elem_size bytes */
void gen_apply_swaps(void* data, uint64_t n, uint32_t elem_size, uint64_t seed, uint64_t stream,
                     uint64_t count) {
  uint64_t b = stream_base(seed, stream), j;
  unsigned char tmp[16];
  unsigned char* d = (unsigned char*)data;
  if (n < 2 || elem_size > 16) return;
  for (j = 0; j < count; j++) {
    uint64_t p = ((word_at(b, 2u * j) >> 32) * n) >> 32;
    uint64_t q = ((word_at(b, 2u * j + 1u) >> 32) * n) >> 32;
    memcpy(tmp, d + p * elem_size, elem_size);
    memcpy(d + p * elem_size, d + q * elem_size, elem_size);
    memcpy(d + q * elem_size, tmp, elem_size);
  }
}

static int cmp_u32(const void* a, const void* b) {
  const uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x > y) - (x < y);
}

/* Concatenated u32 segments, one OpenMP task per segment.  Segment i has
 * sizes[i] keys at offs[i] and kind kinds[i]:
 *   0 uniform on [0, 255]   (high 32 bits & 255, stream 1000 + i)
 *   1 uniform 32-bit        (stream 1000 + i)
 *   2 64 distinct 32-bit values (seed * 7919 + i, stream 1) drawn with
 *     Zipf(1.1) ranks (same seed, stream 2)
 *   3 uniform 32-bit, ascending (libc qsort)
 *   4 uniform 32-bit, descending
 * Returns 0, or -1 when a Zipf table could not be allocated. */
int gen_segments_u32(uint64_t seed, uint32_t nseg, const int64_t* sizes, const int64_t* kinds,
                     const uint64_t* offs, uint32_t* out) {
  int64_t i;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
  for (i = 0; i < (int64_t)nseg; i++) {
    uint32_t* dst = out + offs[i];
    const uint64_t n = (uint64_t)sizes[i];
    const uint64_t st = 1000u + (uint64_t)i;
    uint64_t j;
    switch (kinds[i]) {
      case 0:
        gen_u32(seed, st, n, 255u, dst);
        break;
      case 1:
        gen_u32(seed, st, n, 0xFFFFFFFFu, dst);
        break;
      case 2: {
        uint64_t vals[64];
        uint32_t* idx = (uint32_t*)malloc((n ? n : 1) * sizeof(uint32_t));
        if (!idx) { bad |= 1; break; }
        gen_distinct(seed * 7919u + (uint64_t)i, 1, 64, 32, vals);
        if (gen_zipf_index(seed * 7919u + (uint64_t)i, 2, n, 1.1, 64, idx) != 0) bad |= 1;
        for (j = 0; j < n; j++) dst[j] = (uint32_t)vals[idx[j]];
        free(idx);
        break;
      }
      default:
        gen_u32(seed, st, n, 0xFFFFFFFFu, dst);
        qsort(dst, n, sizeof(uint32_t), cmp_u32);
        if (kinds[i] == 4)
          for (j = 0; j < n / 2; j++) {
            const uint32_t t = dst[j];
            dst[j] = dst[n - 1 - j];
            dst[n - 1 - j] = t;
          }
        break;
    }
  }
  return bad ? -1 : 0;
}
