/*
 * Adaptive Hybrid Sort -- CPU oracle (TEST INFRASTRUCTURE ONLY; see the
 * header for the passages followed and the readings taken).
 *
 * Plain single-threaded C99.  Every sort works on records (mapped key,
 * payload) so that stability and payload movement are explicit.
 */
#include "ahs_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  uint64_t key; /* mapped key */
  uint32_t val; /* payload (or 0) */
} rec_t;

/* ------------------------------------------------------------------------ */
/* Configuration presets (Table II; Sec. III-A; Sec. III-H).                 */
/* ------------------------------------------------------------------------ */
int ref_config_init(ref_config* cfg, int preset) {
  if (!cfg) return REF_E_INVALID_ARG;
  cfg->n_small = 20;       /* n <= 20 -> insertion (Sec. III-A, Table II) */
  cfg->use_model = 0;
  cfg->k_count = 4096;     /* reading R1 */
  cfg->k_radix = 1000000;  /* k > 10^6 (Sec. III-A, Table II) */
  cfg->h_ratio = 0.7;      /* H < 0.7 log2 k (Sec. III-A) */
  cfg->ml_min_n = 1000;    /* predictor for n >= 1000 (Sec. III-H) */
  cfg->k_count_cap = 65536;
  if (preset == 0) return REF_OK;
  if (preset == 1) { cfg->k_count = 1000; return REF_OK; }
  if (preset == 2) { cfg->k_count = 1024; return REF_OK; }
  if (preset == 3) {       /* thresholds recalibrated by eq. (1) (Sec. III-C) */
    cfg->n_small = 48;
    cfg->k_count = 5000;
    return REF_OK;
  }
  return REF_E_INVALID_ARG;
}

/* ------------------------------------------------------------------------ */
/* Key map (reading R11).  Unsigned keys map to themselves.  For IEEE keys a  */
/* set sign bit flips every bit, a clear one sets the sign bit; this orders   */
/* -inf < negatives < -0.0 < +0.0 < positives < +inf as unsigned integers.    */
/* ------------------------------------------------------------------------ */
static int nan32(uint32_t b) {
  return (b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu) != 0u;
}
static int nan64(uint64_t b) {
  return (b & 0x7FF0000000000000ull) == 0x7FF0000000000000ull &&
         (b & 0x000FFFFFFFFFFFFFull) != 0ull;
}

/* Signed keys (the paper's negative-number handling, Listing 7, splits them */
/* into two buckets): as unsigned keys they are v - INT_MIN, computed with    */
/* wrap-around, which is order-preserving.                                    */
int ref_map_keys(int dtype, const void* keys, uint64_t n, uint64_t* mapped,
                 uint64_t* nan_count) {
  uint64_t i, nans = 0;
  if (dtype < REF_U32 || dtype > REF_I64) return REF_E_INVALID_ARG;
  if (n && (!keys || !mapped)) return REF_E_INVALID_ARG;
  for (i = 0; i < n; i++) {
    if (dtype == REF_I32) {
      int32_t v;
      memcpy(&v, (const char*)keys + 4 * i, 4);
      mapped[i] = (uint64_t)((int64_t)v - (int64_t)INT32_MIN);
    } else if (dtype == REF_I64) {
      int64_t v;
      memcpy(&v, (const char*)keys + 8 * i, 8);
      mapped[i] = (uint64_t)v - (uint64_t)INT64_MIN;
    } else if (dtype == REF_U32) {
      mapped[i] = ((const uint32_t*)keys)[i];
    } else if (dtype == REF_U64) {
      mapped[i] = ((const uint64_t*)keys)[i];
    } else if (dtype == REF_F32) {
      uint32_t b;
      memcpy(&b, (const char*)keys + 4 * i, 4);
      if (nan32(b)) nans++;
      mapped[i] = (b & 0x80000000u) ? (uint32_t)~b : (b | 0x80000000u);
    } else {
      uint64_t b;
      memcpy(&b, (const char*)keys + 8 * i, 8);
      if (nan64(b)) nans++;
      mapped[i] = (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
    }
  }
  if (nan_count) *nan_count = nans;
  return nans ? REF_E_NAN : REF_OK;
}

int ref_unmap_keys(int dtype, const uint64_t* mapped, uint64_t n, void* keys) {
  uint64_t i;
  if (dtype < REF_U32 || dtype > REF_I64) return REF_E_INVALID_ARG;
  for (i = 0; i < n; i++) {
    uint64_t m = mapped[i];
    if (dtype == REF_I32) {
      const int32_t v = (int32_t)((int64_t)m + (int64_t)INT32_MIN);
      memcpy((char*)keys + 4 * i, &v, 4);
    } else if (dtype == REF_I64) {
      const uint64_t u = m + (uint64_t)INT64_MIN;
      memcpy((char*)keys + 8 * i, &u, 8);
    } else if (dtype == REF_U32) {
      ((uint32_t*)keys)[i] = (uint32_t)m;
    } else if (dtype == REF_U64) {
      ((uint64_t*)keys)[i] = m;
    } else if (dtype == REF_F32) {
      uint32_t m32 = (uint32_t)m;
      uint32_t b = (m32 & 0x80000000u) ? (m32 & 0x7FFFFFFFu) : ~m32;
      memcpy((char*)keys + 4 * i, &b, 4);
    } else {
      uint64_t b = (m & 0x8000000000000000ull) ? (m & 0x7FFFFFFFFFFFFFFFull) : ~m;
      memcpy((char*)keys + 8 * i, &b, 8);
    }
  }
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Features (Sec. III-A): n, min, max, k = span + 1, and the Shannon entropy  */
/* H = -sum p_i log2 p_i of the key distribution, over at most 65,536 bins    */
/* (reading R3).                                                              */
/* ------------------------------------------------------------------------ */
static int features_of_mapped(const uint64_t* m, uint64_t n, uint32_t* hist,
                              ref_features* f) {
  uint64_t i, mn, mx;
  uint32_t s, nb, b;
  uint32_t* cnt;
  double H = 0.0;

  f->n = n;
  if (n == 0) return REF_OK;
  mn = m[0];
  mx = m[0];
  for (i = 1; i < n; i++) {
    if (m[i] < mn) mn = m[i];
    if (m[i] > mx) mx = m[i];
  }
  f->min_key = mn;
  f->max_key = mx;
  f->span = mx - mn;
  s = 0;
  while ((f->span >> s) > 65535u) s++;
  nb = (uint32_t)(f->span >> s) + 1u;
  f->shift = s;
  f->nbins = nb;
  f->exact = (s == 0) ? 1u : 0u;

  cnt = (uint32_t*)calloc(nb, sizeof(uint32_t));
  if (!cnt) return REF_E_OOM;
  for (i = 0; i < n; i++) cnt[(m[i] - mn) >> s]++;
  for (b = 0; b < nb; b++) {
    if (cnt[b]) {
      double p = (double)cnt[b] / (double)n;
      H -= p * log2(p);
    }
  }
  f->entropy_bits = H;
  f->entropy_ratio = nb > 1 ? H / log2((double)nb) : 0.0;
  if (hist) memcpy(hist, cnt, (size_t)nb * sizeof(uint32_t));
  free(cnt);
  return REF_OK;
}

int ref_features_compute(int dtype, const void* keys, uint64_t n,
                         uint32_t* hist, ref_features* out) {
  uint64_t* m;
  uint64_t nans = 0;
  int st;
  if (!out) return REF_E_INVALID_ARG;
  memset(out, 0, sizeof *out);
  if (dtype < REF_U32 || dtype > REF_I64) return REF_E_INVALID_ARG;
  out->n = n;
  if (n == 0) return REF_OK;
  if (!keys) return REF_E_INVALID_ARG;
  m = (uint64_t*)malloc(n * sizeof(uint64_t));
  if (!m) return REF_E_OOM;
  st = ref_map_keys(dtype, keys, n, m, &nans);
  out->nan_count = nans;
  if (st == REF_OK) st = features_of_mapped(m, n, hist, out);
  free(m);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Learned predictor (Sec. III-H).  Gradient-boosted trees over the inputs    */
/* (n, k, H) with one score per class {COUNTING, RADIX, QUICK}; the class     */
/* with the largest summed score wins, ties to the lower class.               */
/* File format (text):                                                        */
/*   ahs-gbt 1                                                                */
/*   num_class 3                                                              */
/*   base_score <s0> <s1> <s2>                                                */
/*   num_trees <T>                                                            */
/*   then T times:  tree <class> <num_nodes>                                  */
/*                  followed by num_nodes lines, node ids 0..num_nodes-1:     */
/*                    <id> split <feature 0|1|2> <threshold> <left> <right>   */
/*                    <id> leaf <value>                                       */
/* A split goes left when x[feature] < threshold.  Node 0 is the root.        */
/* ------------------------------------------------------------------------ */
typedef struct {
  int is_leaf;
  int feature;
  double threshold;
  int left, right;
  double value;
} ref_node;

typedef struct {
  int cls;
  int nnodes;
  ref_node* nodes;
} ref_tree;

struct ref_model {
  double base[3];
  int ntrees;
  ref_tree* trees;
};

void ref_model_free(ref_model* m) {
  int t;
  if (!m) return;
  if (m->trees) {
    for (t = 0; t < m->ntrees; t++) free(m->trees[t].nodes);
    free(m->trees);
  }
  free(m);
}

int ref_model_load(const char* path, ref_model** out) {
  FILE* fp;
  char word[64];
  int version, ncls, t, i;
  ref_model* m;
  if (!path || !out) return REF_E_INVALID_ARG;
  *out = NULL;
  fp = fopen(path, "r");
  if (!fp) return REF_E_INVALID_ARG;
  m = (ref_model*)calloc(1, sizeof *m);
  if (!m) { fclose(fp); return REF_E_OOM; }
  if (fscanf(fp, "%63s %d", word, &version) != 2 || strcmp(word, "ahs-gbt") || version != 1) goto bad;
  if (fscanf(fp, "%63s %d", word, &ncls) != 2 || strcmp(word, "num_class") || ncls != 3) goto bad;
  if (fscanf(fp, "%63s %lf %lf %lf", word, &m->base[0], &m->base[1], &m->base[2]) != 4 ||
      strcmp(word, "base_score")) goto bad;
  if (fscanf(fp, "%63s %d", word, &m->ntrees) != 2 || strcmp(word, "num_trees") ||
      m->ntrees < 0 || m->ntrees > 100000) goto bad;
  m->trees = (ref_tree*)calloc((size_t)m->ntrees + 1, sizeof(ref_tree));
  if (!m->trees) goto bad;
  for (t = 0; t < m->ntrees; t++) {
    ref_tree* tr = &m->trees[t];
    if (fscanf(fp, "%63s %d %d", word, &tr->cls, &tr->nnodes) != 3 || strcmp(word, "tree") ||
        tr->cls < 0 || tr->cls > 2 || tr->nnodes < 1 || tr->nnodes > 1000000) goto bad;
    tr->nodes = (ref_node*)calloc((size_t)tr->nnodes, sizeof(ref_node));
    if (!tr->nodes) goto bad;
    for (i = 0; i < tr->nnodes; i++) {
      int id;
      ref_node nd;
      memset(&nd, 0, sizeof nd);
      if (fscanf(fp, "%d %63s", &id, word) != 2 || id < 0 || id >= tr->nnodes) goto bad;
      if (!strcmp(word, "split")) {
        if (fscanf(fp, "%d %lf %d %d", &nd.feature, &nd.threshold, &nd.left, &nd.right) != 4) goto bad;
        if (nd.feature < 0 || nd.feature > 2 || nd.left <= id || nd.right <= id ||
            nd.left >= tr->nnodes || nd.right >= tr->nnodes) goto bad;
      } else if (!strcmp(word, "leaf")) {
        nd.is_leaf = 1;
        if (fscanf(fp, "%lf", &nd.value) != 1) goto bad;
      } else {
        goto bad;
      }
      tr->nodes[id] = nd;
    }
  }
  fclose(fp);
  *out = m;
  return REF_OK;
bad:
  fclose(fp);
  ref_model_free(m);
  return REF_E_PARSE;
}

int ref_model_predict(const ref_model* m, const ref_features* f, int* strategy) {
  double x[3], score[3];
  int t, c, best;
  if (!m || !f || !strategy) return REF_E_INVALID_ARG;
  x[0] = (double)f->n;
  x[1] = (double)f->span + 1.0; /* k = max - min + 1 (Sec. III-H) */
  x[2] = f->entropy_bits;
  for (c = 0; c < 3; c++) score[c] = m->base[c];
  for (t = 0; t < m->ntrees; t++) {
    const ref_tree* tr = &m->trees[t];
    int id = 0;
    while (!tr->nodes[id].is_leaf)
      id = (x[tr->nodes[id].feature] < tr->nodes[id].threshold) ? tr->nodes[id].left
                                                                 : tr->nodes[id].right;
    score[tr->cls] += tr->nodes[id].value;
  }
  best = 0;
  for (c = 1; c < 3; c++)
    if (score[c] > score[best]) best = c;
  *strategy = REF_COUNTING + best;
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Decision engine (Sec. III-A FSM, evaluated in the paper's order; Sec.      */
/* III-H: the predictor is consulted for n >= ml_min_n, static rules below).  */
/* ------------------------------------------------------------------------ */
int ref_select(const ref_features* f, const ref_config* cfg,
               const ref_model* model, int* strategy) {
  int s;
  if (!f || !cfg || !strategy || cfg->k_count == 0) return REF_E_INVALID_ARG;
  if (f->n <= cfg->n_small) {
    *strategy = REF_INSERTION;
    return REF_OK;
  }
  if (f->span <= cfg->k_count - 1u) {
    s = REF_COUNTING;
  } else if (f->span >= cfg->k_radix &&
             f->entropy_bits < cfg->h_ratio * log2((double)f->nbins)) {
    s = REF_RADIX;
  } else {
    s = REF_QUICK;
  }
  if (cfg->use_model && f->n >= cfg->ml_min_n) {
    int c;
    if (!model) return REF_E_NO_MODEL;
    ref_model_predict(model, f, &c);
    if (!(c == REF_COUNTING && f->span >= cfg->k_count_cap)) s = c;
  }
  *strategy = s;
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Insertion sort (Sec. III-E, Listing 1): shift while the left neighbour is  */
/* strictly greater, which keeps equal keys in input order.                   */
/* ------------------------------------------------------------------------ */
static void sort_insertion(rec_t* a, uint64_t n) {
  uint64_t i;
  for (i = 1; i < n; i++) {
    rec_t cur = a[i];
    uint64_t j = i;
    while (j > 0 && a[j - 1].key > cur.key) {
      a[j] = a[j - 1];
      j--;
    }
    a[j] = cur;
  }
}

/* ------------------------------------------------------------------------ */
/* Counting sort (Sec. III-F, Listing 2): count occurrences of key - min over */
/* k = span + 1 bins, inclusive prefix sums, then place records scanning      */
/* from the back, decrementing the count, which keeps it stable.              */
/* ------------------------------------------------------------------------ */
static int sort_counting(rec_t* a, uint64_t n, uint64_t mn, uint64_t span) {
  uint64_t k = span + 1u, i, b;
  uint64_t* count;
  rec_t* out;
  count = (uint64_t*)calloc(k, sizeof(uint64_t));
  out = (rec_t*)malloc((n ? n : 1) * sizeof(rec_t));
  if (!count || !out) { free(count); free(out); return REF_E_OOM; }
  for (i = 0; i < n; i++) count[a[i].key - mn]++;
  for (b = 1; b < k; b++) count[b] += count[b - 1];
  for (i = n; i-- > 0;) out[--count[a[i].key - mn]] = a[i];
  memcpy(a, out, n * sizeof(rec_t));
  free(count);
  free(out);
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Radix sort (Sec. III-G, eq. (4)): LSD, base 256, over key - min, with      */
/* d = max(1, ceil(bitlen(span)/8)) digit passes (reading R5).  Each pass is  */
/* a stable distribution of the records into 256 buckets in input order.     */
/* ------------------------------------------------------------------------ */
static int bitlen64(uint64_t x) {
  int b = 0;
  while (x) { b++; x >>= 1; }
  return b;
}

static int sort_radix(rec_t* a, uint64_t n, uint64_t mn, uint64_t span) {
  int d = (bitlen64(span) + 7) / 8, p;
  uint64_t i;
  rec_t *src = a, *dst, *tmp;
  if (d < 1) d = 1;
  tmp = (rec_t*)malloc((n ? n : 1) * sizeof(rec_t));
  if (!tmp) return REF_E_OOM;
  dst = tmp;
  for (p = 0; p < d; p++) {
    uint64_t count[256], start[256], run = 0;
    int b;
    memset(count, 0, sizeof count);
    for (i = 0; i < n; i++) count[((src[i].key - mn) >> (8 * p)) & 255u]++;
    for (b = 0; b < 256; b++) { start[b] = run; run += count[b]; }
    for (i = 0; i < n; i++) dst[start[((src[i].key - mn) >> (8 * p)) & 255u]++] = src[i];
    { rec_t* t = src; src = dst; dst = t; }
  }
  if (src != a) memcpy(a, src, n * sizeof(rec_t));
  free(tmp);
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Quicksort (Sec. III-G.1, Listing 4) with the median-of-three pivot taken   */
/* from the first, middle (floor(len/2)) and last element of the range.  The  */
/* listing's filter partition keeps only x < p and x > p; here the range is   */
/* partitioned out of place into <, ==, > in input order (reading R7), and    */
/* the < and > parts are recursed on through an explicit stack.  A depth      */
/* guard turns adversarial inputs into REF_E_DEPTH instead of running for     */
/* hours.                                                                     */
/* ------------------------------------------------------------------------ */
static uint64_t median3(uint64_t x, uint64_t y, uint64_t z) {
  if (x > y) { uint64_t t = x; x = y; y = t; }
  if (y > z) { uint64_t t = y; y = z; z = t; }
  if (x > y) { uint64_t t = x; x = y; y = t; }
  return y;
}

static int sort_quick(rec_t* a, uint64_t n) {
  typedef struct { uint64_t lo, hi; int depth; } frame_t;
  frame_t* stack;
  int sp = 0, cap = 256, limit;
  rec_t* tmp;
  if (n < 2) return REF_OK;
  limit = 4 * bitlen64(n) + 64;
  tmp = (rec_t*)malloc(n * sizeof(rec_t));
  stack = (frame_t*)malloc((size_t)cap * sizeof(frame_t));
  if (!tmp || !stack) { free(tmp); free(stack); return REF_E_OOM; }
  stack[sp].lo = 0; stack[sp].hi = n; stack[sp].depth = 0; sp++;
  while (sp > 0) {
    frame_t f = stack[--sp];
    uint64_t len = f.hi - f.lo, i, nl = 0, ne = 0, ng = 0, w;
    uint64_t pivot;
    if (len <= 1) continue;
    if (f.depth > limit) { free(tmp); free(stack); return REF_E_DEPTH; }
    pivot = median3(a[f.lo].key, a[f.lo + len / 2].key, a[f.hi - 1].key);
    for (i = f.lo; i < f.hi; i++) {
      if (a[i].key < pivot) nl++;
      else if (a[i].key == pivot) ne++;
      else ng++;
    }
    w = 0;
    for (i = f.lo; i < f.hi; i++) if (a[i].key < pivot) tmp[w++] = a[i];
    for (i = f.lo; i < f.hi; i++) if (a[i].key == pivot) tmp[w++] = a[i];
    for (i = f.lo; i < f.hi; i++) if (a[i].key > pivot) tmp[w++] = a[i];
    memcpy(a + f.lo, tmp, len * sizeof(rec_t));
    if (sp + 2 > cap) {
      frame_t* ns;
      cap *= 2;
      ns = (frame_t*)realloc(stack, (size_t)cap * sizeof(frame_t));
      if (!ns) { free(tmp); free(stack); return REF_E_OOM; }
      stack = ns;
    }
    /* push the larger part first so the smaller one is handled next */
    {
      frame_t lt, gt;
      lt.lo = f.lo; lt.hi = f.lo + nl; lt.depth = f.depth + 1;
      gt.lo = f.lo + nl + ne; gt.hi = f.hi; gt.depth = f.depth + 1;
      if (nl >= ng) { stack[sp++] = lt; stack[sp++] = gt; }
      else { stack[sp++] = gt; stack[sp++] = lt; }
    }
  }
  free(tmp);
  free(stack);
  return REF_OK;
}

/* ------------------------------------------------------------------------ */
/* Whole method (Sec. III intro, Fig. 1): features -> decision -> sort.       */
/* ------------------------------------------------------------------------ */
int ref_sort(int dtype, const void* keys_in, void* keys_out,
             const uint32_t* vals_in, uint32_t* vals_out, uint64_t n,
             int requested, const ref_config* cfg, const ref_model* model,
             int* chosen, ref_features* feats) {
  ref_features f;
  uint64_t *m = NULL, i, nans = 0;
  rec_t* r = NULL;
  int st, strat;

  memset(&f, 0, sizeof f);
  if (chosen) *chosen = REF_AUTO;
  if (feats) memset(feats, 0, sizeof *feats);
  if (dtype < REF_U32 || dtype > REF_I64 || !cfg) return REF_E_INVALID_ARG;
  if (requested < REF_AUTO || requested > REF_INSERTION) return REF_E_INVALID_ARG;
  if ((vals_in == NULL) != (vals_out == NULL)) return REF_E_INVALID_ARG;
  if (n && (!keys_in || !keys_out)) return REF_E_INVALID_ARG;
  f.n = n;

  m = (uint64_t*)malloc((n ? n : 1) * sizeof(uint64_t));
  r = (rec_t*)malloc((n ? n : 1) * sizeof(rec_t));
  if (!m || !r) { st = REF_E_OOM; goto done; }
  st = ref_map_keys(dtype, keys_in, n, m, &nans);
  f.nan_count = nans;
  if (st != REF_OK) goto done;
  st = features_of_mapped(m, n, NULL, &f);
  if (st != REF_OK) goto done;

  if (requested == REF_AUTO) {
    st = ref_select(&f, cfg, model, &strat);
    if (st != REF_OK) goto done;
  } else {
    strat = requested;
    if (strat == REF_COUNTING && n > 0 && f.span >= cfg->k_count_cap) {
      st = REF_E_UNSUPPORTED;
      goto done;
    }
  }

  for (i = 0; i < n; i++) {
    r[i].key = m[i];
    r[i].val = vals_in ? vals_in[i] : 0u;
  }
  if (n > 0) {
    switch (strat) {
      case REF_INSERTION: sort_insertion(r, n); break;
      case REF_COUNTING: st = sort_counting(r, n, f.min_key, f.span); break;
      case REF_RADIX: st = sort_radix(r, n, f.min_key, f.span); break;
      case REF_QUICK: st = sort_quick(r, n); break;
      default: st = REF_E_INVALID_ARG; break;
    }
    if (st != REF_OK) goto done;
  }
  for (i = 0; i < n; i++) m[i] = r[i].key;
  ref_unmap_keys(dtype, m, n, keys_out);
  if (vals_out)
    for (i = 0; i < n; i++) vals_out[i] = r[i].val;
  if (chosen) *chosen = strat;

done:
  if (feats) *feats = f;
  free(m);
  free(r);
  return st;
}
