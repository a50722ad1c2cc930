/*
 * Seeded synthetic record generator (input generator only).
 *
 * This module produces the fixed-length ASCII records that both the GPU sort
 * and the CPU oracle consume.  It holds none of the sorting method's
 * arithmetic: no key encoding, no model, no partitioning.  Every byte is a
 * pure function of (seed, record index), so any range of a data set can be
 * regenerated on demand and the same bytes reach both sides.
 *
 * Random source: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), implemented here from its published
 * definition: 10 rounds of two 32x32->64 multiplies (M0 = 0xD2511F53,
 * M1 = 0xCD9E8D57) with a Weyl key schedule (W0 = 0x9E3779B9,
 * W1 = 0xBB67AE85).
 *
 * Record layout (the paper's benchmark records, Section 7.1): record_bytes
 * bytes, the first key_bytes are the key; everything is printable ASCII
 * 0x20..0x7E.  Counter layout: ctr = {idx_lo, idx_hi, stream, block},
 * key = {seed_lo, seed_hi}.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

enum {
  GEN_UNIFORM = 0,     /* every key byte iid uniform over 0x20..0x7E            */
  GEN_NORMAL_HOT = 1,  /* key bytes: discrete normal over the rank; hot keys    */
  GEN_ZIPF_FIRST = 2,  /* first byte Zipf over the rank, other bytes uniform    */
  GEN_MIX = 3,         /* per record: UNIFORM with prob mix_p, else NORMAL_HOT  */
  GEN_STAIRCASE = 4    /* uniform records whose leading bytes are replaced by an
                          entry of a 128-row prefix table chosen by
                          floor(log2(idx)) mod 128 (Section 7.1's description of
                          the skewed benchmark data, table drawn from our RNG)  */
};

enum { STREAM_KEY = 0, STREAM_PAYLOAD = 1, STREAM_CHOICE = 2, STREAM_HOT = 3,
       STREAM_JOBS = 4, STREAM_STAIR = 5 };

typedef struct {
  uint32_t kind;
  uint32_t record_bytes;
  uint32_t key_bytes;
  uint32_t embed_idx;      /* nonzero: payload bytes [key_bytes, key_bytes+10) hold
                              the record index as 10 decimal digits              */
  uint64_t seed;
  double mean_rank;        /* GEN_NORMAL_HOT: mean character rank (48 = 'P')      */
  double sigma;            /* GEN_NORMAL_HOT: std-dev in characters (6)           */
  double hot_fraction;     /* GEN_NORMAL_HOT: probability a record takes a hot key */
  uint32_t n_hot;          /* GEN_NORMAL_HOT: number of hot keys (1000)           */
  uint32_t stair_bytes;    /* GEN_STAIRCASE: prefix length (6)                    */
  double zipf_s;           /* GEN_ZIPF_FIRST: exponent (1.1)                      */
  double mix_p;            /* GEN_MIX: probability of a uniform record (0.5)      */
} gen_spec;

static inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[1] = (uint32_t)p1;
    c[3] = (uint32_t)p0;
    c[0] = n0;
    c[2] = n2;
  }
}

/* Exposed for the known-answer test of the generator's RNG. */
void gen_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  philox(c, key[0], key[1]);
  memcpy(out, c, sizeof c);
}

static inline void draw(uint64_t seed, uint64_t idx, uint32_t stream, uint32_t block, uint32_t out[4]) {
  out[0] = (uint32_t)idx;
  out[1] = (uint32_t)(idx >> 32);
  out[2] = stream;
  out[3] = block;
  philox(out, (uint32_t)seed, (uint32_t)(seed >> 32));
}

/* Inverse-CDF table over the 95 character ranks: thr[r] = round(2^32 * P(R <= r)),
 * thr[94] = 2^32.  A draw u maps to the smallest r with u < thr[r]. */
typedef struct { uint64_t thr[95]; } rank_law;

static void law_from_weights(const double w[95], rank_law* law) {
  double tot = 0.0;
  for (int r = 0; r < 95; ++r) tot += w[r];
  double acc = 0.0;
  for (int r = 0; r < 95; ++r) {
    acc += w[r];
    double t = ldexp(acc / tot, 32);
    uint64_t v = (uint64_t)llround(t);
    if (v > (1ull << 32)) v = 1ull << 32;
    law->thr[r] = v;
  }
  law->thr[94] = 1ull << 32;
}

static void law_normal(double mean, double sigma, rank_law* law) {
  double w[95];
  for (int r = 0; r < 95; ++r) {
    double z = (r - mean) / sigma;
    w[r] = exp(-0.5 * z * z);
  }
  law_from_weights(w, law);
}

static void law_zipf(double s, rank_law* law) {
  double w[95];
  for (int r = 0; r < 95; ++r) w[r] = pow((double)(r + 1), -s);
  law_from_weights(w, law);
}

static inline uint8_t rank_from_law(const rank_law* law, uint32_t u) {
  int lo = 0, hi = 94;          /* smallest r with u < thr[r] */
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if ((uint64_t)u < law->thr[mid]) hi = mid; else lo = mid + 1;
  }
  return (uint8_t)lo;
}

static inline uint8_t uniform_char(uint32_t u) { return (uint8_t)(0x20 + (uint32_t)(((uint64_t)u * 95u) >> 32)); }

/* key bytes from STREAM_KEY for record/hot index idx under a law (NULL = uniform) */
static void make_key(uint64_t seed, uint64_t idx, uint32_t stream, const rank_law* law0,
                     const rank_law* law_rest, uint8_t* key, uint32_t key_bytes) {
  uint32_t u[4];
  for (uint32_t b = 0; b < key_bytes; ++b) {
    if ((b & 3) == 0) draw(seed, idx, stream, b >> 2, u);
    uint32_t v = u[b & 3];
    const rank_law* law = b == 0 ? law0 : law_rest;
    key[b] = law ? (uint8_t)(0x20 + rank_from_law(law, v)) : uniform_char(v);
  }
}

static void make_payload(uint64_t seed, uint64_t idx, uint8_t* p, uint32_t nbytes) {
  uint32_t u[4];
  for (uint32_t b = 0; b < nbytes; ++b) {
    if ((b & 15) == 0) draw(seed, idx, STREAM_PAYLOAD, b >> 4, u);
    uint32_t byte = (u[(b >> 2) & 3] >> (8 * (b & 3))) & 0xFFu;
    p[b] = (uint8_t)(0x20 + ((byte * 95u) >> 8));
  }
}

/* Fill out[0 .. count*record_bytes) with records start .. start+count-1. */
int gen_records(const gen_spec* sp, uint64_t start, uint64_t count, uint8_t* out) {
  if (!sp || !out || sp->record_bytes == 0 || sp->key_bytes == 0 || sp->key_bytes > sp->record_bytes)
    return 1;
  if (sp->embed_idx && sp->record_bytes < sp->key_bytes + 10) return 1;
  if (sp->kind > GEN_STAIRCASE) return 1;
  const uint32_t R = sp->record_bytes, K = sp->key_bytes;
  rank_law normal, zipf;
  law_normal(sp->mean_rank, sp->sigma, &normal);
  law_zipf(sp->zipf_s, &zipf);
  const uint32_t n_hot = sp->n_hot ? sp->n_hot : 1;
  const uint32_t stair_rows = 128;
  const uint32_t sb = sp->stair_bytes < K ? sp->stair_bytes : K;

#pragma omp parallel for schedule(static, 4096)
  for (int64_t t = 0; t < (int64_t)count; ++t) {
    uint64_t idx = start + (uint64_t)t;
    uint8_t* rec = out + (uint64_t)t * R;
    uint32_t ch[4];
    draw(sp->seed, idx, STREAM_CHOICE, 0, ch);
    uint32_t kind = sp->kind;
    if (kind == GEN_MIX)
      kind = ((double)ch[2] < sp->mix_p * 4294967296.0) ? GEN_UNIFORM : GEN_NORMAL_HOT;
    if (kind == GEN_UNIFORM || kind == GEN_STAIRCASE) {
      make_key(sp->seed, idx, STREAM_KEY, NULL, NULL, rec, K);
    } else if (kind == GEN_ZIPF_FIRST) {
      make_key(sp->seed, idx, STREAM_KEY, &zipf, NULL, rec, K);
    } else {
      if ((double)ch[0] < sp->hot_fraction * 4294967296.0) {
        uint64_t h = ((uint64_t)ch[1] * n_hot) >> 32;
        make_key(sp->seed, h, STREAM_HOT, &normal, &normal, rec, K);
      } else {
        make_key(sp->seed, idx, STREAM_KEY, &normal, &normal, rec, K);
      }
    }
    if (kind == GEN_STAIRCASE && idx > 0) {
      uint32_t lg = 63 - (uint32_t)__builtin_clzll(idx);
      uint32_t row = lg % stair_rows;
      uint8_t pre[16];
      make_key(sp->seed, row, STREAM_STAIR, NULL, NULL, pre, sb);
      memcpy(rec, pre, sb);
    }
    make_payload(sp->seed, idx, rec + K, R - K);
    if (sp->embed_idx) {
      uint64_t v = idx;
      for (int d = 9; d >= 0; --d) { rec[K + d] = (uint8_t)('0' + v % 10); v /= 10; }
    }
  }
  return 0;
}

/* Job sizes of a batch: n_j = round(exp(U[ln lo, ln hi])), one Philox draw per job. */
int gen_job_sizes(uint64_t seed, uint32_t n_jobs, uint64_t lo, uint64_t hi, uint64_t* out) {
  if (!out || lo == 0 || hi < lo) return 1;
  double a = log((double)lo), b = log((double)hi);
  for (uint32_t j = 0; j < n_jobs; ++j) {
    uint32_t u[4];
    draw(seed, j, STREAM_JOBS, 0, u);
    double x = a + (b - a) * ((double)u[0] / 4294967296.0);
    uint64_t n = (uint64_t)llround(exp(x));
    if (n < lo) n = lo;
    if (n > hi) n = hi;
    out[j] = n;
  }
  return 0;
}

/* The rank law thresholds, exported so tests can check the law's shape. */
void gen_rank_law(uint32_t which, double a, double b, uint64_t thr[95]) {
  rank_law law;
  if (which == 0) law_normal(a, b, &law); else law_zipf(a, &law);
  memcpy(thr, law.thr, sizeof law.thr);
}
