/*
 * ORACLE -- test infrastructure only.
 *
 * Plain, slow, obviously correct CPU implementation of what the GPU sort
 * computes.  Only the test suite, the smoke check and the benchmark's CPU
 * baseline may load this file's library; the product path never does.  It
 * shares no code with the HIP library: its own RNG, its own key encoding, its
 * own model fit and evaluation, its own sort.
 *
 * Parts and the passages they follow (Kristo & Kraska, "Parallel External
 * Sorting of ASCII Records Using Learned Models"):
 *
 *  - oracle_sort_*: the problem itself.  Records are ordered by their leading
 *    key bytes in memcmp byte order (Section 7.1, "Methodology"); records with
 *    equal keys keep their input order (the paper is silent on ties; we read
 *    them as stable).  Written as the definition: sort record indices with a
 *    comparator (memcmp on the key, then index) using libc qsort, then gather.
 *    The comparator is a total order, so the result is unique.
 *  - oracle_e8: the base-95 key encoding of Section 4 on the first 8 key
 *    bytes, value = sum_i (byte_i - 32) * 95^(7-i).  Bytes outside 0x20..0x7E
 *    are not covered by the paper; we saturate: from the first such byte on,
 *    every digit is 0 (byte < 0x20) or 94 (byte > 0x7E), which keeps the code
 *    non-decreasing in memcmp order for every byte string.
 *  - oracle_sample_*: the training sample of Section 3.1 -- 1% of the input,
 *    at most 10M keys (Section 6), at least 1024 (our floor for tiny inputs),
 *    never more than n.  Positions are stratified: sample s is drawn uniformly
 *    from [floor(s*n/S), floor((s+1)*n/S)) with a Philox4x32-10 draw
 *    (Salmon et al., SC'11) keyed by the seed.
 *  - oracle_fit_rmi / oracle_rmi_bucket: the two-level RMI CDF model of
 *    Section 3.1 (a root linear model picks one of L leaf linear models; the
 *    leaf predicts the CDF scaled to B buckets) made monotone so the
 *    partitions satisfy Equation 1.  Root: least squares in FP64 of L*rank/S
 *    on the sorted sample, slope clamped at 0.  Leaf: the linear spline
 *    through its first and last sample (B*rank/S at both ends), output
 *    clamped to the bucket range its own sample ranks span.  Evaluation in
 *    FP32 with explicit fmaf.
 *  - oracle_counts_offsets: partition sizes S_p (Algorithm 1's size vector)
 *    and the output offsets of Section 3.5, write_offset(i) = sum_{k<i} len(P_k)
 *    (exclusive prefix sum, in records).
 *  - oracle_opt_max_bucket: the smallest largest-bucket any monotone bucketing
 *    of the sorted sample's equal-code runs into B buckets can reach (the
 *    "ideal equi-depth size" of the MLP acceptance test).
 *  - checkers: sortedness, an order-independent multiset hash, and the rank of
 *    a (key, index) pair among all records (for sampled checks at full size).
 *
 * Parity pins: see tests/test_oracle_*.py (brute force over permutations, closed
 * forms, library least squares, invariants).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ sort -- */

typedef struct {
  const uint8_t* base;
  uint32_t rec;
  uint32_t key;
} sort_ctx;

static sort_ctx g_ctx; /* qsort has no context argument; the oracle is single-threaded */

static int cmp_key_then_index(const void* pa, const void* pb) {
  uint64_t a = *(const uint64_t*)pa, b = *(const uint64_t*)pb;
  int c = memcmp(g_ctx.base + a * g_ctx.rec, g_ctx.base + b * g_ctx.rec, g_ctx.key);
  if (c != 0) return c;
  return (a > b) - (a < b);
}

/* perm[k] = input index of the record at output position k. */
int oracle_sort_order(const uint8_t* in, uint64_t n, uint32_t rec, uint32_t key, uint64_t* perm) {
  if (n && (!in || !perm)) return 1;
  if (key == 0 || key > rec) return 1;
  for (uint64_t i = 0; i < n; ++i) perm[i] = i;
  g_ctx.base = in;
  g_ctx.rec = rec;
  g_ctx.key = key;
  qsort(perm, n, sizeof(uint64_t), cmp_key_then_index);
  return 0;
}

int oracle_sort_records(const uint8_t* in, uint64_t n, uint32_t rec, uint32_t key, uint8_t* out) {
  if (n == 0) return 0;
  uint64_t* perm = (uint64_t*)malloc(n * sizeof(uint64_t));
  if (!perm) return 2;
  int rc = oracle_sort_order(in, n, rec, key, perm);
  if (rc == 0)
    for (uint64_t k = 0; k < n; ++k) memcpy(out + k * rec, in + perm[k] * rec, rec);
  free(perm);
  return rc;
}

/* -------------------------------------------------------------- checkers -- */

/* For records whose input index is written as 10 decimal digits right after
 * the key (bytes [key, key+10)): the index of the first k where (key, index)
 * of record k is not strictly below that of record k+1, or n when none.  With
 * fixed-width digits the pair compares as the bytes [0, key+10) in memcmp
 * order.  Strictly increasing (key, index) plus the input's multiset of
 * records is the definition of the stable sort, so the two checks together
 * pin the whole output. */
uint64_t oracle_first_unstable(const uint8_t* recs, uint64_t n, uint32_t rec, uint32_t key) {
  uint64_t bad = n;
  int64_t last = (int64_t)n - 1;
#pragma omp parallel for reduction(min : bad)
  for (int64_t k = 0; k < last; ++k)
    if (memcmp(recs + (uint64_t)k * rec, recs + (uint64_t)(k + 1) * rec, key + 10) >= 0 && (uint64_t)k < bad)
      bad = (uint64_t)k;
  return bad;
}

/* Variable-length keys (Section 4's padding rule, read as: a key shorter
 * than the key field is padded with bytes below every byte value).  Record
 * byte len_off holds the length (at most key); the key is the first len bytes
 * of the field.  Keys compare as byte strings: memcmp over the shorter length,
 * then the shorter key first; equal keys by input index. */
typedef struct {
  const uint8_t* base;
  uint32_t rec, key, len_off;
} varlen_ctx;
static varlen_ctx g_vctx;

static int cmp_varlen_then_index(const void* pa, const void* pb) {
  uint64_t a = *(const uint64_t*)pa, b = *(const uint64_t*)pb;
  const uint8_t* ra = g_vctx.base + a * g_vctx.rec;
  const uint8_t* rb = g_vctx.base + b * g_vctx.rec;
  uint32_t la = ra[g_vctx.len_off], lb = rb[g_vctx.len_off];
  if (la > g_vctx.key) la = g_vctx.key;
  if (lb > g_vctx.key) lb = g_vctx.key;
  int c = memcmp(ra, rb, la < lb ? la : lb);
  if (c) return c;
  if (la != lb) return la < lb ? -1 : 1;
  return (a > b) - (a < b);
}

int oracle_sort_order_varlen(const uint8_t* in, uint64_t n, uint32_t rec, uint32_t key, uint32_t len_off,
                             uint64_t* perm) {
  if (!in || !perm || key == 0 || len_off >= rec) return 1;
  for (uint64_t i = 0; i < n; ++i) perm[i] = i;
  g_vctx.base = in;
  g_vctx.rec = rec;
  g_vctx.key = key;
  g_vctx.len_off = len_off;
  qsort(perm, n, sizeof(uint64_t), cmp_varlen_then_index);
  return 0;
}

/* Index of the first k with key(k) > key(k+1), or n when keys never decrease. */
uint64_t oracle_first_unsorted(const uint8_t* recs, uint64_t n, uint32_t rec, uint32_t key) {
  uint64_t bad = n;
  int64_t last = (int64_t)n - 1;
#pragma omp parallel for reduction(min : bad)
  for (int64_t k = 0; k < last; ++k)
    if (memcmp(recs + (uint64_t)k * rec, recs + (uint64_t)(k + 1) * rec, key) > 0 && (uint64_t)k < bad)
      bad = (uint64_t)k;
  return bad;
}

static inline uint64_t mix64(uint64_t z) { /* SplitMix64 output function (Steele et al. 2014) */
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t record_hash(const uint8_t* r, uint32_t rec) {
  uint64_t h = 0xCBF29CE484222325ull; /* FNV-1a 64 */
  for (uint32_t i = 0; i < rec; ++i) { h ^= r[i]; h *= 0x100000001B3ull; }
  return mix64(h);
}

/* Sum mod 2^64 of a 64-bit hash of every record: equal for equal multisets. */
uint64_t oracle_multiset_hash(const uint8_t* recs, uint64_t n, uint32_t rec) {
  uint64_t s = 0;
#pragma omp parallel for reduction(+ : s)
  for (int64_t k = 0; k < (int64_t)n; ++k) s += record_hash(recs + (uint64_t)k * rec, rec);
  return s;
}

/* Number of records i with (key_i, i) < (key, idx): the output position the
 * stable order gives to record idx when key is that record's key. */
uint64_t oracle_rank_of(const uint8_t* in, uint64_t n, uint32_t rec, uint32_t keyb, const uint8_t* key,
                        uint64_t idx) {
  uint64_t cnt = 0;
#pragma omp parallel for reduction(+ : cnt)
  for (int64_t i = 0; i < (int64_t)n; ++i) {
    int c = memcmp(in + (uint64_t)i * rec, key, keyb);
    if (c < 0 || (c == 0 && (uint64_t)i < idx)) cnt++;
  }
  return cnt;
}

/* -------------------------------------------------------------- encoding -- */

uint64_t oracle_e8(const uint8_t* key8) {
  uint64_t v = 0;
  int sat = -1; /* -1: not saturated; else the digit every later position takes */
  for (int i = 0; i < 8; ++i) {
    uint8_t c = key8[i];
    int d;
    if (sat >= 0) d = sat;
    else if (c < 0x20) { sat = 0; d = 0; }
    else if (c > 0x7E) { sat = 94; d = 94; }
    else d = c - 0x20;
    v = v * 95u + (uint64_t)d;
  }
  return v;
}

void oracle_e8_records(const uint8_t* recs, uint64_t n, uint32_t rec, uint64_t* out) {
  for (uint64_t i = 0; i < n; ++i) out[i] = oracle_e8(recs + i * rec);
}

/* ---------------------------------------------------------------- sample -- */

static void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t y0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    uint32_t y1 = (uint32_t)p1;
    uint32_t y2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    uint32_t y3 = (uint32_t)p0;
    c[0] = y0; c[1] = y1; c[2] = y2; c[3] = y3;
  }
}

void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  philox4x32_10(c, key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = c[i];
}

/* S = min(max(ceil(n/100), 1024), 10^7, n) */
uint64_t oracle_sample_size(uint64_t n) {
  uint64_t s = (n + 99) / 100;
  if (s < 1024) s = 1024;
  if (s > 10000000ull) s = 10000000ull;
  if (s > n) s = n;
  return s;
}

/* Stratified positions; counter {s_lo, s_hi, 0x53414D50 ('SAMP'), 0}. */
void oracle_sample_indices(uint64_t n, uint64_t S, uint64_t seed, uint64_t* idx) {
  for (uint64_t s = 0; s < S; ++s) {
    uint64_t lo = s * n / S, hi = (s + 1) * n / S;
    uint32_t c[4] = {(uint32_t)s, (uint32_t)(s >> 32), 0x53414D50u, 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    idx[s] = lo + (((uint64_t)c[0] * (hi - lo)) >> 32);
  }
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

/* Sorted codes of the sampled keys. */
void oracle_sample_codes(const uint8_t* recs, uint64_t n, uint32_t rec, uint64_t S, uint64_t seed,
                         uint64_t* codes) {
  uint64_t* idx = (uint64_t*)malloc(S * sizeof(uint64_t));
  oracle_sample_indices(n, S, seed, idx);
  for (uint64_t s = 0; s < S; ++s) codes[s] = oracle_e8(recs + idx[s] * rec);
  free(idx);
  qsort(codes, S, sizeof(uint64_t), cmp_u64);
}

/* ------------------------------------------------------------- RMI model -- */

static inline float code_to_f32(uint64_t e) { return (float)(double)e; }

/* Root: floor(fmaf(a1, x, a0)) clamped to [0, L-1]. */
uint32_t oracle_rmi_leaf(float a0, float a1, uint32_t L, uint64_t e) {
  float r = floorf(fmaf(a1, code_to_f32(e), a0));
  if (r < 0.0f) return 0;
  if (r > (float)(L - 1)) return L - 1;
  return (uint32_t)r;
}

/* Leaf: floor(fmaf(c, x_l, b)) clamped to [lo, hi], x_l = f32(max(e - base, 0)). */
uint32_t oracle_leaf_bucket(uint64_t base, float c, float b, uint32_t lo, uint32_t hi, uint64_t e) {
  uint64_t d = e >= base ? e - base : 0;
  float y = floorf(fmaf(c, code_to_f32(d), b));
  if (y < (float)lo) return lo;
  if (y > (float)hi) return hi;
  return (uint32_t)y;
}

void oracle_spline_leaves(const uint64_t* e, uint64_t S, const uint64_t* first, uint32_t L, uint32_t B,
                          uint64_t* base, float* c, float* b, uint32_t* lo, uint32_t* hi);

/* Least squares of t on x in FP64 (two-pass, centred).  Returns slope and
 * intercept; the slope is 0 when all x are equal. */
static void lsq(const double* x, const double* t, uint64_t m, double* slope, double* icpt) {
  double sx = 0, st = 0;
  for (uint64_t i = 0; i < m; ++i) { sx += x[i]; st += t[i]; }
  double mx = sx / (double)m, mt = st / (double)m;
  double sxx = 0, sxt = 0;
  for (uint64_t i = 0; i < m; ++i) {
    double dx = x[i] - mx;
    sxx += dx * dx;
    sxt += dx * (t[i] - mt);
  }
  double a = sxx > 0 ? sxt / sxx : 0.0;
  *slope = a;
  *icpt = mt - a * mx;
}

/*
 * Fit on sorted codes e[0..S).  Root target: L*s/S (least squares); leaf j with
 * samples f..g-1: line from (0, B*f/S) to (x(e[g-1]-e[f]), B*(g-1)/S).
 * Outputs: root[0] = a0, root[1] = a1 (FP32), and per leaf j: base, slope c,
 * intercept b (FP32), bucket range lo..hi.
 */
int oracle_fit_rmi(const uint64_t* e, uint64_t S, uint32_t L, uint32_t B, float* root, uint64_t* base,
                   float* c, float* b, uint32_t* lo, uint32_t* hi) {
  if (S == 0 || L == 0 || B == 0) return 1;
  for (uint64_t s = 1; s < S; ++s)
    if (e[s] < e[s - 1]) return 1;
  double* x = (double*)malloc(S * sizeof(double));
  double* t = (double*)malloc(S * sizeof(double));
  if (!x || !t) { free(x); free(t); return 2; }

  for (uint64_t s = 0; s < S; ++s) {
    x[s] = (double)code_to_f32(e[s]);
    t[s] = (double)L * (double)s / (double)S;
  }
  double a1, a0;
  lsq(x, t, S, &a1, &a0);
  if (a1 < 0) { a1 = 0; a0 = (double)L * (double)(S - 1) / (2.0 * (double)S); }
  root[0] = (float)a0;
  root[1] = (float)a1;

  /* first[j] = first rank routed to a leaf >= j; routing is non-decreasing in s */
  uint64_t* first = (uint64_t*)malloc(((uint64_t)L + 1) * sizeof(uint64_t));
  uint64_t s = 0;
  for (uint32_t j = 0; j <= L; ++j) {
    while (s < S && oracle_rmi_leaf(root[0], root[1], L, e[s]) < j) ++s;
    first[j] = s;
  }
  first[L] = S;
  oracle_spline_leaves(e, S, first, L, B, base, c, b, lo, hi);
  free(first);
  free(x);
  free(t);
  return 0;
}

/*
 * Leaves over given sample ranges: leaf j holds the sorted samples
 * first[j] .. first[j+1]-1 (first non-decreasing, first[L] = S).  The line
 * through the leaf's first and last sample, mapped to B*rank/S, clamped to the
 * buckets those ranks span; an empty leaf is the constant next bucket.  Used
 * by both roots: the linear root's ranges come from its routing, the MLP
 * root's from the running maximum of floor(L*y) over the sorted sample.
 */
void oracle_spline_leaves(const uint64_t* e, uint64_t S, const uint64_t* first, uint32_t L, uint32_t B,
                          uint64_t* base, float* c, float* b, uint32_t* lo, uint32_t* hi) {
  for (uint32_t j = 0; j < L; ++j) {
    uint64_t f = first[j], g = first[j + 1];
    if (f >= g) { /* empty leaf: constant at the next non-empty leaf's first bucket */
      uint32_t v = f < S ? (uint32_t)(((uint64_t)B * f) / S) : B - 1;
      base[j] = 0; c[j] = 0.0f; b[j] = (float)v; lo[j] = v; hi[j] = v;
      continue;
    }
    base[j] = e[f];
    /* linear spline through the leaf's first and last sample: the line meets
     * the leaf's own bucket range exactly at both ends */
    double tf = (double)B * (double)f / (double)S;
    double tl = (double)B * (double)(g - 1) / (double)S;
    double span = (double)code_to_f32(e[g - 1] - e[f]);
    double cj = span > 0 ? (tl - tf) / span : 0.0;
    double bj = tf;
    c[j] = (float)cj;
    b[j] = (float)bj;
    lo[j] = (uint32_t)(((uint64_t)B * f) / S);
    uint64_t h = ((uint64_t)B * (g - 1)) / S;
    hi[j] = (uint32_t)(h < B - 1 ? h : B - 1);
  }
}

/* Bucket of every record when the leaf is found from boundary codes: leaf j
 * takes the codes in [bound[j], bound[j+1]), bound[0] = 0, bound[L] beyond
 * every code (binary search for the last bound <= code). */
void oracle_routed_buckets(const uint8_t* recs, uint64_t n, uint32_t rec, const uint64_t* bound, uint32_t L,
                           const uint64_t* base, const float* c, const float* b, const uint32_t* lo,
                           const uint32_t* hi, uint32_t* out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t e = oracle_e8(recs + i * rec);
    uint32_t l0 = 0, h0 = L;
    while (h0 - l0 > 1) {
      uint32_t mid = (l0 + h0) / 2;
      if (bound[mid] <= e) l0 = mid; else h0 = mid;
    }
    out[i] = oracle_leaf_bucket(base[l0], c[l0], b[l0], lo[l0], hi[l0], e);
  }
}

/* Bucket of every record under an RMI. */
void oracle_rmi_buckets(const uint8_t* recs, uint64_t n, uint32_t rec, const float* root, uint32_t L,
                        const uint64_t* base, const float* c, const float* b, const uint32_t* lo,
                        const uint32_t* hi, uint32_t* out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t e = oracle_e8(recs + i * rec);
    uint32_t j = oracle_rmi_leaf(root[0], root[1], L, e);
    out[i] = oracle_leaf_bucket(base[j], c[j], b[j], lo[j], hi[j], e);
  }
}

/* Bucket of every code under an RMI (codes instead of records: the sample). */
void oracle_rmi_buckets_codes(const uint64_t* e, uint64_t n, const float* root, uint32_t L, const uint64_t* base,
                              const float* c, const float* b, const uint32_t* lo, const uint32_t* hi,
                              uint32_t* out) {
  for (uint64_t i = 0; i < n; ++i) {
    uint32_t j = oracle_rmi_leaf(root[0], root[1], L, e[i]);
    out[i] = oracle_leaf_bucket(base[j], c[j], b[j], lo[j], hi[j], e[i]);
  }
}

/* Leaves under a given root (a0, a1): the sorted sample is routed by that
 * root and each leaf takes the spline over the ranks routed to it, as
 * oracle_fit_rmi does after its own least-squares root. */
void oracle_leaves_under_root(const uint64_t* e, uint64_t S, float a0, float a1, uint32_t L, uint32_t B,
                              uint64_t* base, float* c, float* b, uint32_t* lo, uint32_t* hi) {
  uint64_t* first = (uint64_t*)malloc(((uint64_t)L + 1) * sizeof(uint64_t));
  uint64_t s = 0;
  for (uint32_t j = 0; j <= L; ++j) {
    while (s < S && oracle_rmi_leaf(a0, a1, L, e[s]) < j) ++s;
    first[j] = s;
  }
  first[L] = S;
  oracle_spline_leaves(e, S, first, L, B, base, c, b, lo, hi);
  free(first);
}

/* counts[j] = #records with bucket j; offsets[j] = sum_{k<j} counts[k], offsets[B] = n. */
int oracle_counts_offsets(const uint32_t* bucket, uint64_t n, uint32_t B, uint64_t* counts, uint64_t* offsets) {
  for (uint32_t j = 0; j < B; ++j) counts[j] = 0;
  for (uint64_t i = 0; i < n; ++i) {
    if (bucket[i] >= B) return 1;
    counts[bucket[i]]++;
  }
  uint64_t acc = 0;
  for (uint32_t j = 0; j < B; ++j) { offsets[j] = acc; acc += counts[j]; }
  offsets[B] = acc;
  return 0;
}

/* ------------------------------------------------------- ideal max bucket -- */

static int fits(const uint64_t* runs, uint64_t nr, uint64_t cap, uint64_t B) {
  uint64_t used = 1, fill = 0;
  for (uint64_t r = 0; r < nr; ++r) {
    if (runs[r] > cap) return 0;
    if (fill + runs[r] > cap) { used++; fill = 0; if (used > B) return 0; }
    fill += runs[r];
  }
  return 1;
}

/* Smallest C such that the equal-code runs of the sorted codes, kept in order
 * and whole, pack into at most B buckets of at most C each. */
uint64_t oracle_opt_max_bucket(const uint64_t* e, uint64_t S, uint64_t B) {
  if (S == 0) return 0;
  uint64_t* runs = (uint64_t*)malloc(S * sizeof(uint64_t));
  uint64_t nr = 0, len = 1, mx = 0;
  for (uint64_t s = 1; s <= S; ++s) {
    if (s < S && e[s] == e[s - 1]) { len++; continue; }
    runs[nr++] = len;
    if (len > mx) mx = len;
    len = 1;
  }
  uint64_t lo = mx, hi = S; /* greedy packing is optimal for a fixed capacity */
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (fits(runs, nr, mid, B)) hi = mid; else lo = mid + 1;
  }
  free(runs);
  return lo;
}
