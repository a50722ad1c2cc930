// In-bucket sort and concatenation (gfx950): Section 3.4 (sort each partition)
// and Section 3.5 (write it at the exclusive prefix sum of the partition sizes,
// coalescing the records in sorted order).
//
// A bucket's records sit in its region (and possibly the spill area) as
// 128-byte slots: 32-bit input index, record, padding.  Each record gives a
// composite sort key: key bytes 0..11 and then the index, big-endian, so the
// composite order is the key's memcmp order with ties broken by input
// position, and all composites of a bucket differ.  A byte that is equal
// across the whole bucket is never sorted on: every kernel first ORs and ANDs
// the bucket's composites, so an all-equal-key bucket orders its index bytes
// only (early termination on duplicates).
//
//  * bucket_sort_small: buckets of up to 2048 records, one 512-thread block
//    each.  The first 16 bytes of every slot go to LDS; one counting pass on
//    the key's base-95 code, scaled over the bucket's code range into 2048
//    bins (a second, finer one when a bin holds more than 12 entries), then
//    each bin is ordered by the whole composite: ranks counted in parallel up
//    to 64 entries, a one-wave bitonic network up to 256, a whole-bucket LSD
//    radix beyond.  The records are then gathered in sorted
//    order straight into the output (each slot line is read twice: for the
//    key, then for the record).
//  * bucket_sort_lds: buckets of up to 6144 records, the same algorithm with
//    a 13-bit counting digit in one 1024-thread block.
//  * msd_split + seg_sort + big_gather: larger buckets, split by their most
//    significant varying composite byte into pieces the small-bucket sort
//    finishes, then copied out in order (records of at least 64 bytes).
//  * bucket_sort_global: larger buckets of shorter records, stable LSD passes
//    over the varying composite bytes through the bucket's own output range.
//  * long_runs + long_run_sort: keys of 13 to 28 bytes, runs of equal 12-byte
//    prefixes ordered by the rest of the key after the kernels above.
#include "elsar_internal.h"

namespace elsar {

struct BucketRef {      // where the records of one bucket live
  uint32_t n, nr;       // records, records in the region
  uint32_t rs, so;      // region start slot, spill offset
  uint64_t out0;        // first output position
};

__device__ __forceinline__ uint32_t slot_of(const BucketRef& br, uint32_t p, const uint32_t* __restrict__ spill_map,
                                            uint64_t cap_slots) {
  return p < br.nr ? br.rs + p : (uint32_t)cap_slots + spill_map[br.so + (p - br.nr)];
}

__device__ __forceinline__ uint32_t key_tail_mask(uint32_t K) {  // key bytes 8..K-1, big-endian in a word
  uint32_t tb = K - 8;
  return tb == 0 ? 0u : (tb >= 4 ? ~0u : (0xFFFFFFFFu << (32 - 8 * tb)));
}

// Composite sort key of a slot as four words, word 0 most significant: key
// bytes [0, K) then the 4 index bytes, big-endian, zero beyond.  Slot dword 0
// is the index, dwords 1.. the record.
__device__ __forceinline__ uint4 composite_words(uint32_t idx, uint32_t r0, uint32_t r1, uint32_t r2, uint32_t K) {
  uint32_t tb = K - 8;
  uint32_t t = __builtin_bswap32(r2) & key_tail_mask(K);
  uint64_t low = ((uint64_t)t << 32) | ((uint64_t)idx << (32 - 8 * tb));
  return make_uint4(__builtin_bswap32(r0), __builtin_bswap32(r1), (uint32_t)(low >> 32), (uint32_t)low);
}

// The composite of a slot; with variable-length keys (vk != 0) of the
// record's virtual key (virtual_key), K then counting its length byte.
__device__ __forceinline__ uint4 composite(const uint32_t* __restrict__ s, uint32_t K, uint32_t vk) {
  uint32_t r0 = s[1], r1 = s[2], r2 = s[3];
  virtual_key(r0, r1, r2, vk);
  return composite_words(s[0], r0, r1, r2, K);
}

__device__ __forceinline__ uint32_t digit_of(const uint4& c, uint32_t p) {
  uint32_t w = p < 4 ? c.x : (p < 8 ? c.y : (p < 12 ? c.z : c.w));
  return (w >> (24 - 8 * (p & 3))) & 0xFFu;
}

// OR ^ AND of every thread's composite words across the block: the bits that
// differ somewhere in the bucket.
template <uint32_t THREADS>
__device__ uint4 block_diff(uint4 o, uint4 a, uint4* sh_or, uint4* sh_and) {
  const uint32_t w = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    o.x |= __shfl_xor(o.x, off); o.y |= __shfl_xor(o.y, off);
    o.z |= __shfl_xor(o.z, off); o.w |= __shfl_xor(o.w, off);
    a.x &= __shfl_xor(a.x, off); a.y &= __shfl_xor(a.y, off);
    a.z &= __shfl_xor(a.z, off); a.w &= __shfl_xor(a.w, off);
  }
  if (lane_id() == 0) { sh_or[w] = o; sh_and[w] = a; }
  __syncthreads();
  uint4 O = sh_or[0], A = sh_and[0];
  for (uint32_t i = 1; i < THREADS / 64; ++i) {
    uint4 x = sh_or[i], y = sh_and[i];
    O.x |= x.x; O.y |= x.y; O.z |= x.z; O.w |= x.w;
    A.x &= y.x; A.y &= y.y; A.z &= y.z; A.w &= y.w;
  }
  __syncthreads();
  return make_uint4(O.x ^ A.x, O.y ^ A.y, O.z ^ A.z, O.w ^ A.w);
}

// Block-wide min and max of one u64 per thread; every thread gets both.
template <uint32_t THREADS>
__device__ void block_min_max_u64(uint64_t& mn, uint64_t& mx, uint64_t* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t a = shfl_xor_u64(mn, off), b = shfl_xor_u64(mx, off);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 0) { sh[2 * w] = mn; sh[2 * w + 1] = mx; }
  __syncthreads();
  mn = sh[0];
  mx = sh[1];
  for (uint32_t i = 1; i < THREADS / 64; ++i) {
    mn = sh[2 * i] < mn ? sh[2 * i] : mn;
    mx = sh[2 * i + 1] > mx ? sh[2 * i + 1] : mx;
  }
  __syncthreads();
}

// Bit p set when composite byte p (0..15) varies.
__device__ __forceinline__ uint32_t vary_mask(const uint4& d) {
  uint32_t vary = 0;
  for (uint32_t p = 0; p < 16; ++p) vary |= (uint32_t)(digit_of(d, p) != 0) << p;
  return vary;
}

template <uint32_t THREADS>
__device__ uint32_t varying_bytes(uint4 o, uint4 a, uint4* sh_or, uint4* sh_and) {
  return vary_mask(block_diff<THREADS>(o, a, sh_or, sh_and));
}

// Exclusive scan over the 256 digits of per-wave counts wc[w][d] -> start
// offsets wc[w][d] in digit-major, wave-minor order.  Needs THREADS >= 256.
template <uint32_t WAVES>
__device__ void digit_wave_offsets(uint32_t (*wc)[256], uint32_t* tot) {
  if (threadIdx.x < 256) {
    uint32_t d = threadIdx.x, run = 0;
    for (uint32_t w = 0; w < WAVES; ++w) {
      uint32_t c = wc[w][d];
      wc[w][d] = run;
      run += c;
    }
    uint32_t v = run;  // inclusive scan of the digit totals over the first 4 waves
    for (int off = 1; off < 64; off <<= 1) {
      uint32_t x = __shfl_up(v, off);
      if (lane_id() >= (uint32_t)off) v += x;
    }
    if (lane_id() == 63) tot[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t add = 0;
    for (uint32_t i = 0; i < (threadIdx.x >> 6); ++i) add += tot[i];
    uint32_t excl = v - run + add;
    for (uint32_t w = 0; w < WAVES; ++w) wc[w][d] += excl;
  } else {
    __syncthreads();
  }
}

// One stable counting pass of perm[cur][0..n) on the digit dg(e) of each entry
// e; the result goes to perm[cur ^ 1].  Each wave ranks a contiguous segment
// of ROUNDS*64 positions in order, so ties keep their order.
template <uint32_t CAP, uint32_t THREADS, typename Digit>
__device__ void lsd_pass(uint16_t (*perm)[CAP], uint32_t cur, uint32_t n, uint32_t (*wc)[256], uint32_t* tot,
                         Digit dg) {
  constexpr uint32_t WAVES = THREADS / 64;
  constexpr uint32_t ROUNDS = CAP / THREADS;
  const uint32_t w = threadIdx.x >> 6;
  for (uint32_t i = threadIdx.x; i < WAVES * 256; i += THREADS) (&wc[0][0])[i] = 0;
  __syncthreads();
  uint32_t dv[ROUNDS], lc[ROUNDS];
  uint16_t ev[ROUNDS];
#pragma unroll
  for (uint32_t r = 0; r < ROUNDS; ++r) {
    uint32_t i = w * (ROUNDS * 64) + r * 64 + lane_id();
    bool valid = i < n;
    uint16_t e = valid ? perm[cur][i] : 0;
    uint32_t d = valid ? dg(e) : 0u;
    uint64_t peers = match_digit8(d, valid);
    uint32_t rank = __popcll(peers & lanemask_lt());
    uint32_t prev = valid ? wc[w][d] : 0u;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) wc[w][d] = prev + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
    dv[r] = d;
    lc[r] = prev + rank;
    ev[r] = e;
  }
  __syncthreads();
  digit_wave_offsets<WAVES>(wc, tot);
  __syncthreads();
#pragma unroll
  for (uint32_t r = 0; r < ROUNDS; ++r) {
    uint32_t i = w * (ROUNDS * 64) + r * 64 + lane_id();
    if (i < n) perm[cur ^ 1][wc[w][dv[r]] + lc[r]] = ev[r];
  }
  __syncthreads();
}

// ------------------------------------------- buckets of up to 2048 records --
constexpr uint32_t kSmThreads = 512;
constexpr uint32_t kSmWaves = kSmThreads / 64;
constexpr uint32_t kSmCap = kSmallCap;
constexpr uint32_t kSmBits = 11;     // counting-sort digit: 2048 bins of the bucket's code range
constexpr uint32_t kSmGroup = 7;     // gathered chunks in flight per thread
constexpr uint32_t kRunMax = 64;     // longest bin ordered by counted ranks
constexpr uint32_t kWaveSortMax = 256;  // longest bin a wave sorts (bitonic); longer ones: LSD over the bucket

// LDS writes of a wave visible to all its lanes (compiler ordering; one
// wave's LDS operations complete in order)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Steps after the digits: the digit of entry p is in perm[1][p] (2^BITS bins,
// non-decreasing in the composite).  A counting pass on the digit, then the
// whole composite (less) orders each bin: ranks counted in parallel (one
// thread per entry) up to kRunMax entries, a bitonic network (one wave, in its
// own kWaveSortMax entries of perm[1]) up to kWaveSortMax, and stable LSD passes over every
// varying composite byte (byte_of(entry, position)) of the bucket when some
// bin is longer still (keys clustered at a finer scale than the digit
// resolves).  bins: 2^BITS counters, also the LSD passes' per-wave counters.
// Returns the perm buffer that holds the sorted order.
//
// With a position function (pos(entry): the scaled value whose floor is the
// entry's digit, non-decreasing in the key), a bucket with a bin of more than
// kRefineMin entries is counted a second time on a finer digit: bin b's m
// entries, at [s, s + m) after the first pass, get the sub-bins s +
// floor(m * (pos - b)), by where each lies within the bin's own stretch of
// the scale.  The sub-bins refine the bins, so their order stays the key's;
// keys clustered within a bin (the skewed law's per-byte peaks) then meet far
// fewer others of their sub-bin in the rank counting below.
struct NoPos {
  static constexpr bool enabled = false;
  __device__ double operator()(uint32_t) const { return 0.0; }
};
constexpr uint32_t kRefineMin = 12;

template <uint32_t CAP, uint32_t THREADS, uint32_t BITS, typename Less, typename ByteOf, typename Pos = NoPos>
__device__ __forceinline__ uint32_t bin_sort_core(uint32_t n, uint32_t vary, uint16_t (*perm)[CAP], uint32_t* bins,
                                                  uint32_t* sh_scan, uint32_t* tot, Less less, ByteOf byte_of,
                                                  Pos pos = Pos()) {
  constexpr uint32_t WAVES = THREADS / 64, NB = 1u << BITS;
  static_assert(WAVES * 256 <= NB, "the bins double as the LSD counters");
  static_assert(WAVES * kWaveSortMax <= CAP, "a private bitonic area per wave in perm[1]");
  static_assert(!Pos::enabled || CAP <= NB, "the sub-bins of a refined count are positions below n");
  const uint32_t tid = threadIdx.x;
  uint16_t* dig = perm[1];
  auto counting_pass = [&]() {  // bins zeroed: entries to perm[0] by digit; bins[b] is then the end of bin b
    __syncthreads();
    for (uint32_t p = tid; p < n; p += THREADS) atomicAdd(&bins[dig[p]], 1u);
    __syncthreads();
    {  // exclusive scan of the bins: PER contiguous per thread
      constexpr uint32_t PER = NB / THREADS;
      uint32_t c[PER], sum = 0;
#pragma unroll
      for (uint32_t i = 0; i < PER; ++i) { c[i] = bins[tid * PER + i]; sum += c[i]; }
      uint32_t total;
      uint32_t run = block_exclusive_scan<uint32_t, THREADS>(sum, sh_scan, &total);
#pragma unroll
      for (uint32_t i = 0; i < PER; ++i) { bins[tid * PER + i] = run; run += c[i]; }
    }
    __syncthreads();
    for (uint32_t p = tid; p < n; p += THREADS) perm[0][atomicAdd(&bins[dig[p]], 1u)] = (uint16_t)p;
    __syncthreads();
  };
  counting_pass();
  if constexpr (Pos::enabled) {
    bool crowded = false;
    for (uint32_t b = tid; b < NB; b += THREADS) crowded |= bins[b] - (b ? bins[b - 1] : 0u) > kRefineMin;
    if (__syncthreads_or(crowded)) {
      constexpr uint32_t AR = CAP / THREADS;
      static_assert(CAP % THREADS == 0, "whole rounds of entries");
      uint16_t sub[AR];
#pragma unroll
      for (uint32_t i = 0; i < AR; ++i) {
        const uint32_t e = tid + i * THREADS;
        sub[i] = 0;
        if (e < n) {
          const uint32_t b = dig[e];
          const uint32_t s0 = b ? bins[b - 1] : 0u, m = bins[b] - s0;
          double f = pos(e) - (double)b;
          f = f < 0.0 ? 0.0 : f;
          uint32_t k = (uint32_t)(f * (double)m);
          sub[i] = (uint16_t)(s0 + (k < m ? k : m - 1));
        }
      }
      __syncthreads();  // every bin bound is read
#pragma unroll
      for (uint32_t i = 0; i < AR; ++i) {
        const uint32_t e = tid + i * THREADS;
        if (e < n) dig[e] = sub[i];
      }
      for (uint32_t b = tid; b < NB; b += THREADS) bins[b] = 0;
      counting_pass();
    }
  }
  // bins[b] is now the end of bin b; the start is the end of bin b-1
  __shared__ uint16_t wave_bins[CAP / (kRunMax + 1) + 1];  // bins for the waves
  __shared__ uint32_t n_wave_bins;
  if (tid == 0) n_wave_bins = 0;
  __syncthreads();
  bool long_bin = false;
  for (uint32_t b = tid; b < NB; b += THREADS) {  // bins[b] is the end of bin b
    const uint32_t m = bins[b] - (b ? bins[b - 1] : 0u);
    if (m > kRunMax) {
      if (m > kWaveSortMax) long_bin = true;
      else wave_bins[atomicAdd(&n_wave_bins, 1u)] = (uint16_t)b;
    }
  }
  long_bin = __syncthreads_or(long_bin);
  uint32_t cur = 0;
  if (!long_bin) {
    // the bin of each of this thread's positions (start, size), read while
    // the digits are still in perm[1]
    constexpr uint32_t AR = CAP / THREADS;
    static_assert(CAP % THREADS == 0, "whole rounds of positions");
    uint32_t ext[AR];
#pragma unroll
    for (uint32_t i = 0; i < AR; ++i) {
      const uint32_t x = tid + i * THREADS;
      ext[i] = 0;
      if (x < n) {
        const uint32_t d = dig[perm[0][x]];
        const uint32_t b0 = d ? bins[d - 1] : 0u;
        ext[i] = (b0 << 16) | (bins[d] - b0);
      }
    }
    __syncthreads();
    // one wave per bin of kRunMax+1 .. kWaveSortMax entries: bitonic network
    // over the next power of two, padded with a sentinel above every entry
    const uint32_t w = tid >> 6, lane = tid & 63u;
    uint16_t* sc = perm[1] + w * kWaveSortMax;
    const uint32_t nw = n_wave_bins;
    for (uint32_t i = w; i < nw; i += WAVES) {
      const uint32_t b = wave_bins[i];
      const uint32_t s0 = b ? bins[b - 1] : 0u, m = bins[b] - s0;
      uint32_t P = 64;
      while (P < m) P <<= 1;
      for (uint32_t x = lane; x < P; x += 64) sc[x] = x < m ? perm[0][s0 + x] : (uint16_t)0xFFFFu;
      wave_lds_sync();
      for (uint32_t k = 2; k <= P; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
          for (uint32_t x = lane; x < P; x += 64) {
            const uint32_t y = x ^ j;
            if (y > x) {
              const uint16_t a = sc[x], c = sc[y];
              // a > c, with the sentinel above every entry
              const bool gt = a == 0xFFFFu ? c != 0xFFFFu : (c != 0xFFFFu && less(c, a));
              if (gt == ((x & k) == 0)) {
                sc[x] = c;
                sc[y] = a;
              }
            }
          }
          wave_lds_sync();
        }
      }
      for (uint32_t x = lane; x < m; x += 64) perm[0][s0 + x] = sc[x];
      wave_lds_sync();
    }
    __syncthreads();
    // bins of up to kRunMax entries: every entry's rank is the number of
    // entries of its bin below it (one thread per entry, all bins at once);
    // the entries go to perm[1] at bin start + rank, the longer bins (already
    // in order) to the same positions
#pragma unroll
    for (uint32_t i = 0; i < AR; ++i) {
      const uint32_t x = tid + i * THREADS;
      if (x < n) {
        const uint32_t b0 = ext[i] >> 16, m = ext[i] & 0xFFFFu;
        const uint16_t e = perm[0][x];
        uint32_t dest = x;
        if (m <= kRunMax) {
          uint32_t rank = 0;
          for (uint32_t y = b0; y < b0 + m; ++y) rank += less(perm[0][y], e) ? 1u : 0u;
          dest = b0 + rank;
        }
        perm[1][dest] = e;
      }
    }
    __syncthreads();
    cur = 1;
  } else {  // stable LSD over every varying composite byte
    auto wc = reinterpret_cast<uint32_t(*)[256]>(bins);
    for (int pb = 15; pb >= 0; --pb) {
      if (!((vary >> pb) & 1u)) continue;
      lsd_pass<CAP, THREADS>(perm, cur, n, wc, tot, [&](uint32_t e) { return byte_of(e, (uint32_t)pb); });
      cur ^= 1;
    }
  }
  return cur;
}

// The position of a digit taken from a 64-bit source value scaled over the
// bucket's range: (src(entry) - min) * scale.
template <typename Src>
struct ScaledPos {
  static constexpr bool enabled = true;
  Src src;
  uint64_t lo;
  double scale;
  __device__ double operator()(uint32_t e) const { return (double)(src(e) - lo) * scale; }
};
template <typename Src>
__device__ __forceinline__ ScaledPos<Src> scaled_pos(Src src, uint64_t lo, double scale) {
  return ScaledPos<Src>{src, lo, scale};
}

// The small-bucket instance: composites as four word arrays cw[0..3][entry].
template <typename Pos = NoPos>
__device__ __forceinline__ uint32_t small_sort_core(uint32_t n, uint32_t vary, uint32_t (*cw)[kSmCap],
                                                    uint16_t (*perm)[kSmCap], uint32_t* bins, uint32_t* sh_scan,
                                                    uint32_t* tot, Pos pos = Pos()) {
  auto less = [&](uint32_t x, uint32_t y) -> bool {
    if (cw[0][x] != cw[0][y]) return cw[0][x] < cw[0][y];
    if (cw[1][x] != cw[1][y]) return cw[1][x] < cw[1][y];
    if (cw[2][x] != cw[2][y]) return cw[2][x] < cw[2][y];
    return cw[3][x] < cw[3][y];
  };
  auto byte_of = [&](uint32_t e, uint32_t pb) -> uint32_t { return (cw[pb >> 2][e] >> (24 - 8 * (pb & 3))) & 0xFFu; };
  return bin_sort_core<kSmCap, kSmThreads, kSmBits>(n, vary, perm, bins, sh_scan, tot, less, byte_of, pos);
}

template <uint32_t RW>  // record dwords
__device__ __forceinline__ void bucket_sort_small_body(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map, const uint4* __restrict__ slots,
    uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t K, uint32_t* __restrict__ out, uint32_t B,
    uint32_t vk, uint32_t bid, uint32_t nblk) {
  constexpr uint32_t SC = slot_bytes_for(RW * 4) / 16;  // 16-byte chunks per slot
  constexpr uint32_t LC = (RW + 1 + 3) / 4;             // chunks holding the index or record bytes
  constexpr uint32_t AR = kSmCap / kSmThreads;          // entries per thread
  __shared__ uint32_t cw[4][kSmCap];                    // composite words of every entry
  __shared__ uint16_t perm[2][kSmCap];
  __shared__ uint32_t bins[1u << kSmBits];              // also the LSD fallback's per-wave counters
  __shared__ uint4 sh_or[kSmWaves], sh_and[kSmWaves];
  __shared__ uint32_t sh_scan[kSmThreads / 64 + 1];
  __shared__ uint64_t sh_mm[2 * kSmWaves];
  __shared__ uint32_t tot[4];
  static_assert((1u << kSmBits) == kSmWaves * 256, "bins double as the LSD counters");
  const uint32_t tid = threadIdx.x;
  const uint32_t j = bid;
  if (j >= B) return;
  // the bucket's header words, loaded together before the test on its size
  // (the empty asm statement takes them as operands, so the compiler cannot
  // defer the other loads past the test: one round trip instead of three)
  BucketRef br;
  br.n = counts[j];
  const uint32_t cap = caps[j];
  br.rs = rstart[j];
  br.so = spill_off[j];
  br.out0 = offsets[j];
  __asm__ volatile("" ::"s"(cap), "s"(br.rs), "s"(br.so), "s"(br.out0));
  if (br.n == 0 || br.n > kSmCap) return;
  br.nr = br.n < cap ? br.n : cap;
  const uint32_t n = br.n;

  // 1. the first 16 bytes of every slot: index and key.  The slots are found
  //    first and the loads go out together, unconditionally (positions past
  //    the bucket's end reload its last slot): a load under "p < n" was
  //    waited for inside its branch, which made the four loads of a thread
  //    four round trips.
  uint32_t sl[AR];
#pragma unroll
  for (uint32_t i = 0; i < AR; ++i) {
    const uint32_t p = tid + i * kSmThreads;
    sl[i] = slot_of(br, p < n ? p : n - 1, spill_map, cap_slots);
  }
  uint4 v[AR];
#pragma unroll
  for (uint32_t i = 0; i < AR; ++i) v[i] = slots[(uint64_t)sl[i] * SC];
  if (vk) {
#pragma unroll
    for (uint32_t i = 0; i < AR; ++i) virtual_key(v[i].y, v[i].z, v[i].w, vk);
  }
  uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
  uint64_t cmin = ~0ull, cmax = 0;  // base-95 codes of the first 8 key bytes
#pragma unroll
  for (uint32_t i = 0; i < AR; ++i) {
    uint32_t p = tid + i * kSmThreads;
    if (p < n) {
      uint4 c = composite_words(v[i].x, v[i].y, v[i].z, v[i].w, K);
      cw[0][p] = c.x; cw[1][p] = c.y; cw[2][p] = c.z; cw[3][p] = c.w;
      o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
      a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
      uint64_t e = key_code(v[i].y, v[i].z);
      cmin = e < cmin ? e : cmin;
      cmax = e > cmax ? e : cmax;
    }
  }
  // bits that vary across the bucket (syncs; the entries are visible afterwards)
  const uint4 diff = block_diff<kSmThreads>(o, a, sh_or, sh_and);
  const uint32_t vary = vary_mask(diff);
  block_min_max_u64<kSmThreads>(cmin, cmax, sh_mm);
  uint32_t cur = 0;
  if (n == 1) {
    if (tid == 0) perm[0][0] = 0;
  } else {
    // 2. one counting pass on a digit of the key's base-95 code scaled over the
    //    bucket's code range: (code - min) * 2^kSmBits / (max - min + 1).  It is
    //    a non-decreasing function of the key, and near uniform over an
    //    equi-depth bucket.  Entries with equal digits are then ordered by the
    //    whole composite.
    const double scale = (double)(1u << kSmBits) / ((double)(cmax - cmin) + 1.0);
    uint16_t* dig = perm[1];  // the digits, until a fallback needs the buffer
    for (uint32_t i = tid; i < (1u << kSmBits); i += kSmThreads) bins[i] = 0;
#pragma unroll
    for (uint32_t i = 0; i < AR; ++i) {
      uint32_t p = tid + i * kSmThreads;
      if (p < n) {
        uint64_t e = key_code(v[i].y, v[i].z);
        uint32_t d = (uint32_t)((double)(e - cmin) * scale);
        dig[p] = (uint16_t)(d < (1u << kSmBits) ? d : (1u << kSmBits) - 1);
      }
    }
    auto code_of = [&](uint32_t e) -> uint64_t {
      return key_code(__builtin_bswap32(cw[0][e]), __builtin_bswap32(cw[1][e]));
    };
    cur = small_sort_core(n, vary, cw, perm, bins, sh_scan, tot, scaled_pos(code_of, cmin, scale));
  }
  __syncthreads();
  // 3. gather through LDS: the records of sorted positions [r0, r0 + kStage)
  //    are assembled in the composite area (free once the order is known),
  //    then that stretch of the output goes out as whole 128-byte lines of
  //    16-byte nontemporal stores, its partial lines at both ends as dword
  //    stores.  The output is never read back here; whole-line nontemporal
  //    writes keep it from displacing, in L2, the slot lines that other
  //    blocks have fetched for their keys and are about to gather.  The slot
  //    loads are nontemporal too: this is the line's last use.
  uint32_t* stage = &cw[0][0];
  constexpr uint32_t kStage = (4 * kSmCap) / RW;  // records per round
  for (uint32_t r0 = 0; r0 < n; r0 += kStage) {
    const uint32_t m = n - r0 < kStage ? n - r0 : kStage;
    const uint32_t nq = m * LC;
    __syncthreads();  // the composites, or the previous round's stretch, are read
    for (uint32_t q0 = 0; q0 < nq; q0 += kSmGroup * kSmThreads) {
      u32x4 g[kSmGroup];
#pragma unroll
      for (uint32_t i = 0; i < kSmGroup; ++i) {  // kSmGroup loads in flight per thread
        uint32_t q = q0 + tid + i * kSmThreads;
        uint32_t qq = q < nq ? q : nq - 1;  // clamped: no branch around the loads
        uint32_t k = qq / LC, c = qq - k * LC;
        g[i] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(slots) +
                                          (uint64_t)slot_of(br, perm[cur][r0 + k], spill_map, cap_slots) * SC + c);
      }
#pragma unroll
      for (uint32_t i = 0; i < kSmGroup; ++i) {
        uint32_t q = q0 + tid + i * kSmThreads;
        if (q < nq) {
          uint32_t k = q / LC, c = q - k * LC;
#pragma unroll
          for (uint32_t t = 0; t < 4; ++t) {
            uint32_t sd = 4 * c + t;  // slot dword: 0 is the index, 1..RW the record
            if (sd >= 1 && sd <= RW) stage[k * RW + sd - 1] = g[i][t];
          }
        }
      }
    }
    __syncthreads();
    const uint64_t gb = (br.out0 + r0) * RW;  // first output dword of the stretch
    const uint32_t total = m * RW;
    uint32_t head = (uint32_t)((32u - (uint32_t)(gb & 31u)) & 31u);  // dwords up to a 128-byte boundary
    if (head > total) head = total;
    const uint32_t lines = (total - head) / 32;
    if (tid < head) out[gb + tid] = stage[tid];
    for (uint32_t v = tid; v < lines * 8; v += kSmThreads) {
      const uint32_t s0 = head + 4 * v;
      u32x4 x;
      x[0] = stage[s0];
      x[1] = stage[s0 + 1];
      x[2] = stage[s0 + 2];
      x[3] = stage[s0 + 3];
      __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(out + gb + head) + v);
    }
    for (uint32_t t = head + lines * 32 + tid; t < total; t += kSmThreads) out[gb + t] = stage[t];
  }
}

template <uint32_t RW>
__global__ __launch_bounds__(kSmThreads) void bucket_sort_small_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map, const uint4* __restrict__ slots,
    uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t K, uint32_t* __restrict__ out, uint32_t B,
    uint32_t vk) {
  bucket_sort_small_body<RW>(counts, caps, rstart, spill_off, spill_map, slots, cap_slots, offsets, K, out, B, vk, blockIdx.x, gridDim.x);
}

// ------------------------------------------- buckets of up to 6144 records --
// The small-bucket algorithm at a larger scale: one counting pass on a
// 12-bit (up to 3072 entries) or 13-bit digit of the base-95 code over the
// bucket's code range, then the per-bin orderings of bin_sort_core.  Two
// instances take the mid list: buckets of up to kMidLoCap records (listed from
// the start of mid_list, 76 KB of LDS, two 512-thread blocks per CU) and the
// larger ones (listed from its end, 157 KB, one 1024-thread block per CU).
constexpr uint32_t kMidThreads = 1024;  // 16 waves: the one block a CU holds (157 KB of LDS)
constexpr uint32_t kMidLoThreads = 512;

template <uint32_t CAP, uint32_t THREADS>
__device__ __forceinline__ void bucket_sort_lds_body(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    bool from_end, uint32_t B, PartHeader* __restrict__ reset, uint32_t vk, uint32_t bid,
    uint32_t nblk) {
  constexpr uint32_t kMidBits = CAP <= kMidLoCap ? 12u : 13u;
  // the first kernel of the larger buckets' chain clears the split's counters
  // and the list of buckets the equal-key kernel passes on, so every call of
  // the chain on a partition is the same
  if (reset && bid == 0 && threadIdx.x < 5) {
    if (threadIdx.x < 4) reset->seg_n[threadIdx.x] = 0;
    else reset->n_big2 = 0;
  }
  constexpr uint32_t WAVES = THREADS / 64;
  static_assert(CAP % THREADS == 0, "cap is whole rounds");
  __shared__ uint4 ent[CAP];
  __shared__ uint16_t perm[2][CAP];
  __shared__ uint32_t bins[1u << kMidBits];
  __shared__ uint4 sh_or[WAVES], sh_and[WAVES];
  __shared__ uint64_t sh_mm[2 * WAVES];
  __shared__ uint32_t sh_scan[WAVES + 1];
  __shared__ uint32_t tot[4];
  auto less = [&](uint32_t x, uint32_t y) -> bool {
    const uint4 a = ent[x], b = ent[y];
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    if (a.z != b.z) return a.z < b.z;
    return a.w < b.w;
  };
  auto byte_of = [&](uint32_t e, uint32_t pb) -> uint32_t { return digit_of(ent[e], pb); };
  const uint32_t W = slot_bytes_for(RW * 4) / 4;  // slot stride in dwords
  const uint32_t nitems = list ? *list_n : B;
  for (uint32_t it = bid; it < nitems; it += nblk) {
    const uint32_t j = list ? list[from_end ? B - 1 - it : it] : it;
    // the header words together, before the test on the count (as in the
    // small-bucket kernel)
    BucketRef br;
    br.n = counts[j];
    const uint32_t cap = caps[j];
    br.rs = rstart[j];
    br.so = spill_off[j];
    br.out0 = offsets[j];
    __asm__ volatile("" ::"s"(cap), "s"(br.rs), "s"(br.so), "s"(br.out0));
    if (br.n == 0 || br.n > CAP) continue;
    br.nr = br.n < cap ? br.n : cap;
    // 1. load the entries (every thread's slot heads in flight together, past
    //    the bucket's end its last slot again), and the range of their
    //    base-95 codes
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    uint64_t cmin = ~0ull, cmax = 0;
    constexpr uint32_t NL = (CAP / THREADS) % 3 == 0 ? 3 : 4;  // heads per thread in flight
    for (uint32_t p0 = 0; p0 < br.n; p0 += NL * THREADS) {
     uint32_t sl[NL];
#pragma unroll
     for (uint32_t i = 0; i < NL; ++i) {
      const uint32_t p = p0 + threadIdx.x + i * THREADS;
      sl[i] = slot_of(br, p < br.n ? p : br.n - 1, spill_map, cap_slots);
     }
     uint4 hv[NL];
#pragma unroll
     for (uint32_t i = 0; i < NL; ++i) hv[i] = *reinterpret_cast<const uint4*>(slots + (uint64_t)sl[i] * W);
#pragma unroll
     for (uint32_t i = 0; i < NL; ++i) {
      const uint32_t p = p0 + threadIdx.x + i * THREADS;
      if (p < br.n) {
        uint32_t r0 = hv[i].y, r1 = hv[i].z, r2 = hv[i].w;
        virtual_key(r0, r1, r2, vk);
        const uint4 c = composite_words(hv[i].x, r0, r1, r2, K);
        ent[p] = c;
        o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
        a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
        const uint64_t e = key_code(r0, r1);
        cmin = e < cmin ? e : cmin;
        cmax = e > cmax ? e : cmax;
      }
     }
    }
    const uint4 diff = block_diff<THREADS>(o, a, sh_or, sh_and);  // syncs
    const uint32_t vary = vary_mask(diff);
    block_min_max_u64<THREADS>(cmin, cmax, sh_mm);
    // 2. the digit (code - min) * 2^kMidBits / (max - min + 1), non-decreasing
    //    in the key, then the bin sorts
    const double scale = (double)(1u << kMidBits) / ((double)(cmax - cmin) + 1.0);
    for (uint32_t i = threadIdx.x; i < (1u << kMidBits); i += THREADS) bins[i] = 0;
    for (uint32_t p = threadIdx.x; p < br.n; p += THREADS) {
      const uint4 c = ent[p];
      const uint64_t e = key_code(__builtin_bswap32(c.x), __builtin_bswap32(c.y));
      const uint32_t d = (uint32_t)((double)(e - cmin) * scale);
      perm[1][p] = (uint16_t)(d < (1u << kMidBits) ? d : (1u << kMidBits) - 1);
    }
    auto code_of = [&](uint32_t e) -> uint64_t {
      return key_code(__builtin_bswap32(ent[e].x), __builtin_bswap32(ent[e].y));
    };
    const uint32_t cur = bin_sort_core<CAP, THREADS, kMidBits>(br.n, vary, perm, bins, sh_scan, tot, less, byte_of,
                                                               scaled_pos(code_of, cmin, scale));
    __syncthreads();
    // 3. copy records in sorted order to the output through LDS, as in the
    //    small-bucket kernel: a stretch of records assembled in the entry
    //    area (free once the order is known), then whole 128-byte lines of
    //    nontemporal 16-byte stores, dword stores at the stretch's ends
    const uint32_t SC = W / 4, LC = (RW + 1 + 3) / 4;
    const u32x4* s4 = reinterpret_cast<const u32x4*>(slots);
    uint32_t* stage = reinterpret_cast<uint32_t*>(ent);
    const uint32_t kStage = (4 * CAP) / RW;  // records per round
    for (uint32_t r0 = 0; r0 < br.n; r0 += kStage) {
      const uint32_t m = br.n - r0 < kStage ? br.n - r0 : kStage;
      const uint32_t nq = m * LC;
      __syncthreads();  // the entries, or the previous round's stretch, are read
      for (uint32_t q0 = 0; q0 < nq; q0 += kSmGroup * THREADS) {
        u32x4 g[kSmGroup];
#pragma unroll
        for (uint32_t i = 0; i < kSmGroup; ++i) {
          const uint32_t q = q0 + threadIdx.x + i * THREADS;
          const uint32_t qq = q < nq ? q : nq - 1;
          const uint32_t k = qq / LC, c = qq - k * LC;
          g[i] = __builtin_nontemporal_load(s4 + (uint64_t)slot_of(br, perm[cur][r0 + k], spill_map, cap_slots) * SC +
                                            c);
        }
#pragma unroll
        for (uint32_t i = 0; i < kSmGroup; ++i) {
          const uint32_t q = q0 + threadIdx.x + i * THREADS;
          if (q < nq) {
            const uint32_t k = q / LC, c = q - k * LC;
#pragma unroll
            for (uint32_t t = 0; t < 4; ++t) {
              const uint32_t sd = 4 * c + t;  // slot dword: 0 is the index, 1..RW the record
              if (sd >= 1 && sd <= RW) stage[k * RW + sd - 1] = g[i][t];
            }
          }
        }
      }
      __syncthreads();
      const uint64_t gb = (br.out0 + r0) * RW;  // first output dword of the stretch
      const uint32_t total = m * RW;
      uint32_t head = (uint32_t)((32u - (uint32_t)(gb & 31u)) & 31u);
      if (head > total) head = total;
      const uint32_t lines = (total - head) / 32;
      if (threadIdx.x < head) out[gb + threadIdx.x] = stage[threadIdx.x];
      for (uint32_t v = threadIdx.x; v < lines * 8; v += THREADS) {
        const uint32_t s0 = head + 4 * v;
        u32x4 x;
        x[0] = stage[s0];
        x[1] = stage[s0 + 1];
        x[2] = stage[s0 + 2];
        x[3] = stage[s0 + 3];
        __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(out + gb + head) + v);
      }
      for (uint32_t t = head + lines * 32 + threadIdx.x; t < total; t += THREADS) out[gb + t] = stage[t];
    }
    __syncthreads();
  }
}

template <uint32_t CAP, uint32_t THREADS>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(CAP == kMidLoCap ? 4 : 1))) void bucket_sort_lds_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    bool from_end, uint32_t B, PartHeader* __restrict__ reset, uint32_t vk) {
  bucket_sort_lds_body<CAP, THREADS>(counts, caps, rstart, spill_off, spill_map, slots, cap_slots, offsets, RW, K, out, list, list_n, from_end, B, reset, vk, blockIdx.x, gridDim.x);
}

// ------------------------------------------ big buckets of one repeated key --
// A bucket above the mid cap whose keys are all equal -- a heavily repeated
// key, which the equi-depth roots give a bucket of its own -- is in order
// once its records are in input order.  One block per bucket:
//  1. a probe: the keys of 64 records spread over the bucket, so that a
//     bucket of different keys is handed on after 64 reads, not n;
//  2. the 16-byte head of every slot: the key words (checked equal across
//     the bucket) and the input index, kept in LDS;
//  3. the positions ordered by index: a counting pass on a digit of the index
//     scaled over the bucket's index range, then bin_sort_core's per-bin
//     orderings (the indices of a hot key are spread over the input, so the
//     bins hold a few entries each);
//  4. the records copied in that order through an LDS stage, as in the other
//     bucket sorts.
// A bucket whose keys differ, or one above kEqCap records, goes on the list
// the general split takes (list2).
constexpr uint32_t kEqCap = 16384;
constexpr uint32_t kEqThreads = 1024;
constexpr uint32_t kEqBits = 12;  // counting digit: 4096 bins of the index range

constexpr uint32_t kEqLoads = 2;  // slot heads per thread in flight

__device__ __forceinline__ void equal_keys_body(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    uint32_t* __restrict__ list2, uint32_t* __restrict__ list2_n, uint32_t vk, uint32_t bid, uint32_t nblk) {
  constexpr uint32_t WAVES = kEqThreads / 64;
  __shared__ uint32_t idx[kEqCap];  // input index of each position; after the sort, the stage
  __shared__ uint16_t perm[2][kEqCap];
  __shared__ uint32_t bins[1u << kEqBits];
  __shared__ uint4 sh_or[WAVES], sh_and[WAVES];
  __shared__ uint32_t sh_scan[WAVES + 1];
  __shared__ uint64_t sh_mm[2 * WAVES];
  __shared__ uint32_t tot[4];
  __shared__ uint32_t probe_vary;
  const uint32_t tid = threadIdx.x;
  const uint32_t W = slot_bytes_for(RW * 4) / 4;  // slot stride in dwords
  const uint32_t SC = W / 4, LC = (RW + 1 + 3) / 4;
  const uint32_t key_mask = (1u << K) - 1u;        // composite bytes of the key
  const uint32_t nitems = *list_n;
  for (uint32_t it = bid; it < nitems; it += nblk) {
    const uint32_t j = list[it];
    BucketRef br;
    br.n = counts[j];
    const uint32_t n = br.n;
    const uint32_t cap = caps[j];
    br.nr = n < cap ? n : cap;
    br.rs = rstart[j];
    br.so = spill_off[j];
    br.out0 = offsets[j];
    // 1. the probe (wave 0)
    if (tid < 64) {
      const uint32_t p = (uint32_t)(((uint64_t)tid * n) / 64);
      uint4 c = composite(slots + (uint64_t)slot_of(br, p, spill_map, cap_slots) * W, K, vk), o = c, a = c;
      for (int off = 32; off > 0; off >>= 1) {
        o.x |= __shfl_xor(o.x, off); o.y |= __shfl_xor(o.y, off);
        o.z |= __shfl_xor(o.z, off); o.w |= __shfl_xor(o.w, off);
        a.x &= __shfl_xor(a.x, off); a.y &= __shfl_xor(a.y, off);
        a.z &= __shfl_xor(a.z, off); a.w &= __shfl_xor(a.w, off);
      }
      if (tid == 0) probe_vary = vary_mask(make_uint4(o.x ^ a.x, o.y ^ a.y, o.z ^ a.z, o.w ^ a.w)) & key_mask;
    }
    __syncthreads();
    const bool probe_differs = probe_vary != 0;
    __syncthreads();  // probe_vary is read before the next bucket's probe writes it
    if (probe_differs || n > kEqCap) {
      if (tid == 0) list2[atomicAdd(list2_n, 1u)] = j;
      continue;
    }
    // 2. heads: the key words (OR / AND across the bucket), the indices and
    //    their range; kEqLoads heads per thread in flight together
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    uint64_t imin = ~0ull, imax = 0;
    for (uint32_t p0 = 0; p0 < n; p0 += kEqLoads * kEqThreads) {
      uint32_t sl[kEqLoads];
#pragma unroll
      for (uint32_t i = 0; i < kEqLoads; ++i) {
        const uint32_t p = p0 + tid + i * kEqThreads;
        sl[i] = slot_of(br, p < n ? p : n - 1, spill_map, cap_slots);  // past the end: the last slot again
      }
      uint4 hv[kEqLoads];
#pragma unroll
      for (uint32_t i = 0; i < kEqLoads; ++i) hv[i] = *reinterpret_cast<const uint4*>(slots + (uint64_t)sl[i] * W);
#pragma unroll
      for (uint32_t i = 0; i < kEqLoads; ++i) {
        const uint32_t p = p0 + tid + i * kEqThreads;
        if (p < n) {
          uint32_t r0 = hv[i].y, r1 = hv[i].z, r2 = hv[i].w;
          virtual_key(r0, r1, r2, vk);
          const uint4 c = composite_words(hv[i].x, r0, r1, r2, K);
          o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
          a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
          const uint32_t x = hv[i].x;
          idx[p] = x;
          imin = x < imin ? x : imin;
          imax = x > imax ? x : imax;
        }
      }
    }
    const uint32_t vary = vary_mask(block_diff<kEqThreads>(o, a, sh_or, sh_and));  // syncs
    if (vary & key_mask) {  // the keys differ after all: the general split takes the bucket
      if (tid == 0) list2[atomicAdd(list2_n, 1u)] = j;
      continue;
    }
    block_min_max_u64<kEqThreads>(imin, imax, sh_mm);
    // 3. positions in index order: the digit (index - min) * 2^kEqBits / (max - min + 1)
    const double scale = (double)(1u << kEqBits) / ((double)(imax - imin) + 1.0);
    for (uint32_t i = tid; i < (1u << kEqBits); i += kEqThreads) bins[i] = 0;
    for (uint32_t p = tid; p < n; p += kEqThreads) {
      const uint32_t d = (uint32_t)((double)(idx[p] - (uint32_t)imin) * scale);
      perm[1][p] = (uint16_t)(d < (1u << kEqBits) ? d : (1u << kEqBits) - 1);
    }
    const uint32_t span = (uint32_t)(imax ^ imin);  // index bytes that can differ (big-endian positions 0..3)
    uint32_t ivary = 0;
    for (uint32_t pb = 0; pb < 4; ++pb) ivary |= (uint32_t)((span >> (24 - 8 * pb)) != 0) << pb;
    auto less = [&](uint32_t x, uint32_t y) -> bool { return idx[x] < idx[y]; };
    auto byte_of = [&](uint32_t e, uint32_t pb) -> uint32_t { return (idx[e] >> (24 - 8 * pb)) & 0xFFu; };
    const uint32_t cur = bin_sort_core<kEqCap, kEqThreads, kEqBits>(n, ivary, perm, bins, sh_scan, tot, less, byte_of);
    __syncthreads();
    // 4. the records in that order, through the stage (the index area, free now)
    uint32_t* stage = idx;
    const uint32_t kStage = kEqCap / RW;  // records per round
    const u32x4* s4 = reinterpret_cast<const u32x4*>(slots);
    for (uint32_t r0 = 0; r0 < n; r0 += kStage) {
      const uint32_t m = n - r0 < kStage ? n - r0 : kStage;
      const uint32_t nq = m * LC;
      __syncthreads();  // the previous round's stretch is read
      for (uint32_t q0 = 0; q0 < nq; q0 += kSmGroup * kEqThreads) {
        u32x4 g[kSmGroup];
#pragma unroll
        for (uint32_t i = 0; i < kSmGroup; ++i) {
          const uint32_t q = q0 + tid + i * kEqThreads;
          const uint32_t qq = q < nq ? q : nq - 1;
          const uint32_t k = qq / LC, c = qq - k * LC;
          g[i] = __builtin_nontemporal_load(s4 + (uint64_t)slot_of(br, perm[cur][r0 + k], spill_map, cap_slots) * SC +
                                            c);
        }
#pragma unroll
        for (uint32_t i = 0; i < kSmGroup; ++i) {
          const uint32_t q = q0 + tid + i * kEqThreads;
          if (q < nq) {
            const uint32_t k = q / LC, c = q - k * LC;
#pragma unroll
            for (uint32_t t = 0; t < 4; ++t) {
              const uint32_t sd = 4 * c + t;  // slot dword: 0 is the index, 1..RW the record
              if (sd >= 1 && sd <= RW) stage[k * RW + sd - 1] = g[i][t];
            }
          }
        }
      }
      __syncthreads();
      const uint64_t gb = (br.out0 + r0) * RW;  // first output dword of the stretch
      const uint32_t total = m * RW;
      uint32_t head = (uint32_t)((32u - (uint32_t)(gb & 31u)) & 31u);
      if (head > total) head = total;
      const uint32_t lines = (total - head) / 32;
      if (tid < head) out[gb + tid] = stage[tid];
      for (uint32_t v = tid; v < lines * 8; v += kEqThreads) {
        const uint32_t s0 = head + 4 * v;
        u32x4 x;
        x[0] = stage[s0];
        x[1] = stage[s0 + 1];
        x[2] = stage[s0 + 2];
        x[3] = stage[s0 + 3];
        __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(out + gb + head) + v);
      }
      for (uint32_t t = head + lines * 32 + tid; t < total; t += kEqThreads) out[gb + t] = stage[t];
    }
    __syncthreads();  // the stage is read before the next bucket's indices overwrite it
  }
}

__global__ __launch_bounds__(kEqThreads) void equal_keys_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    uint32_t* __restrict__ list2, uint32_t* __restrict__ list2_n, uint32_t vk) {
  equal_keys_body(counts, caps, rstart, spill_off, spill_map, slots, cap_slots, offsets, RW, K, out, list, list_n,
                  list2, list2_n, vk, blockIdx.x, gridDim.x);
}

// ------------------------------------------------ buckets above the LDS cap --
constexpr uint32_t kBigThreads = 1024;
constexpr uint32_t kBigWaves = kBigThreads / 64;
constexpr uint32_t kBigRounds = 4;
constexpr uint32_t kBigTile = kBigThreads * kBigRounds;

// 20-byte entries (4 composite words + slot) at 4-byte alignment.
__device__ __forceinline__ void put_entry(uint32_t* buf, uint32_t k, const uint4& c, uint32_t slot) {
  uint32_t* p = buf + 5ull * k;
  p[0] = c.x; p[1] = c.y; p[2] = c.z; p[3] = c.w; p[4] = slot;
}
__device__ __forceinline__ uint4 get_key(const uint32_t* buf, uint32_t k) {
  const uint32_t* p = buf + 5ull * k;
  return make_uint4(p[0], p[1], p[2], p[3]);
}

// LDS of the stable LSD passes over 20-byte entries.
struct LsdShared {
  uint32_t wc[kBigWaves][256];  // per wave and digit: count, then output offset
  uint32_t run[256];            // per digit: output position of the tile's first entry
  uint32_t hist[256];
  uint32_t tot[4];
};

// Stable LSD radix passes, least significant byte first, over the composite
// bytes set in `vary` (positions below nb) of n 20-byte entries (4 big-endian
// key words + a payload word), alternating between cur and nxt; one block of
// kBigThreads.  Returns the buffer that holds the sorted entries.
__device__ uint32_t* lsd_entries(uint32_t* cur, uint32_t* nxt, uint32_t n, uint32_t vary, uint32_t nb,
                                 LsdShared& sh) {
  const uint32_t w = threadIdx.x >> 6;
  for (int pbyte = (int)nb - 1; pbyte >= 0; --pbyte) {
    if (!((vary >> pbyte) & 1u)) continue;
    if (threadIdx.x < 256) sh.hist[threadIdx.x] = 0;
    __syncthreads();
    for (uint32_t p = threadIdx.x; p < n; p += kBigThreads) atomicAdd(&sh.hist[digit_of(get_key(cur, p), pbyte)], 1u);
    __syncthreads();
    if (threadIdx.x < 256) {  // exclusive scan of hist -> run
      uint32_t v = sh.hist[threadIdx.x], x = v;
      for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane_id() >= (uint32_t)off) x += y;
      }
      if (lane_id() == 63) sh.tot[threadIdx.x >> 6] = x;
      __syncthreads();
      uint32_t add = 0;
      for (uint32_t i = 0; i < (threadIdx.x >> 6); ++i) add += sh.tot[i];
      sh.run[threadIdx.x] = x - v + add;
    } else {
      __syncthreads();
    }
    __syncthreads();
    for (uint32_t t0 = 0; t0 < n; t0 += kBigTile) {
      for (uint32_t i = threadIdx.x; i < kBigWaves * 256; i += kBigThreads) (&sh.wc[0][0])[i] = 0;
      __syncthreads();
      uint32_t dg[kBigRounds], lc[kBigRounds];
#pragma unroll
      for (uint32_t r = 0; r < kBigRounds; ++r) {
        uint32_t i = t0 + w * (kBigRounds * 64) + r * 64 + lane_id();
        bool valid = i < n;
        uint32_t d = valid ? digit_of(get_key(cur, i), pbyte) : 0u;
        uint64_t peers = match_digit8(d, valid);
        uint32_t rank = __popcll(peers & lanemask_lt());
        uint32_t prev = valid ? sh.wc[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) sh.wc[w][d] = prev + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        dg[r] = d;
        lc[r] = prev + rank;
      }
      __syncthreads();
      // per digit: tile count and wave offsets; then global position = run + offset
      if (threadIdx.x < 256) {
        uint32_t d = threadIdx.x, s = 0;
        for (uint32_t ww = 0; ww < kBigWaves; ++ww) {
          uint32_t c = sh.wc[ww][d];
          sh.wc[ww][d] = s + sh.run[d];
          s += c;
        }
        sh.hist[d] = s;  // this tile's count of digit d
      }
      __syncthreads();
#pragma unroll
      for (uint32_t r = 0; r < kBigRounds; ++r) {
        uint32_t i = t0 + w * (kBigRounds * 64) + r * 64 + lane_id();
        if (i < n) {
          const uint32_t* src = cur + 5ull * i;
          uint32_t dpos = sh.wc[w][dg[r]] + lc[r];
          uint32_t* dst = nxt + 5ull * dpos;
          dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2]; dst[3] = src[3]; dst[4] = src[4];
        }
      }
      __syncthreads();
      if (threadIdx.x < 256) sh.run[threadIdx.x] += sh.hist[threadIdx.x];
      __syncthreads();
    }
    uint32_t* t = cur;
    cur = nxt;
    nxt = t;
  }
  return cur;
}

__device__ __forceinline__ void bucket_sort_global_body(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    uint32_t vk, uint32_t bid,
    uint32_t nblk) {
  __shared__ LsdShared lsd;
  __shared__ uint4 sh_or[kBigWaves], sh_and[kBigWaves];
  __shared__ uint32_t chunk_slot[kBigTile];
  const uint32_t W = slot_bytes_for(RW * 4) / 4;  // slot stride in dwords
  const uint32_t nitems = *list_n;
  for (uint32_t it = bid; it < nitems; it += nblk) {
    const uint32_t j = list[it];
    BucketRef br;
    br.n = counts[j];
    const uint32_t cap = caps[j];
    br.nr = br.n < cap ? br.n : cap;
    br.rs = rstart[j];
    br.so = spill_off[j];
    br.out0 = offsets[j];
    uint32_t* o_dw = out + br.out0 * RW;                  // R*n bytes = RW*n dwords
    uint32_t* buf0 = o_dw + (uint64_t)(RW - 10) * br.n;  // (R-40)*n bytes in
    uint32_t* buf1 = o_dw + (uint64_t)(RW - 5) * br.n;   // (R-20)*n bytes in
    // 1. which composite bytes vary
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint32_t p = threadIdx.x; p < br.n; p += kBigThreads) {
      uint4 c = composite(slots + (uint64_t)slot_of(br, p, spill_map, cap_slots) * W, K, vk);
      o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
      a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
    }
    uint32_t vary = varying_bytes<kBigThreads>(o, a, sh_or, sh_and);
    const uint32_t nb = K + 4;
    uint32_t passes = __popc(vary & ((1u << nb) - 1u));
    // the last pass must land in buf1
    uint32_t* cur = (passes & 1u) ? buf0 : buf1;
    uint32_t* nxt = (passes & 1u) ? buf1 : buf0;
    for (uint32_t p = threadIdx.x; p < br.n; p += kBigThreads) {
      uint32_t sl = slot_of(br, p, spill_map, cap_slots);
      put_entry(cur, p, composite(slots + (uint64_t)sl * W, K, vk), sl);
    }
    __syncthreads();
    // 2. stable LSD passes through global memory
    cur = lsd_entries(cur, nxt, br.n, vary, nb, lsd);
    // 3. copy records in sorted order; entry k sits at or after byte R*(k+1)
    //    of the range, so a chunk's entries are read before its records land.
    for (uint32_t k0 = 0; k0 < br.n; k0 += kBigTile) {
      uint32_t m = br.n - k0 < kBigTile ? br.n - k0 : kBigTile;
      for (uint32_t i = threadIdx.x; i < m; i += kBigThreads) chunk_slot[i] = cur[5ull * (k0 + i) + 4];
      __syncthreads();
      const uint32_t total = m * RW;
      for (uint32_t f = threadIdx.x; f < total; f += kBigThreads) {
        uint32_t k = f / RW, d = f - k * RW;
        o_dw[(uint64_t)k0 * RW + f] = slots[(uint64_t)chunk_slot[k] * W + d + 1];
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kBigThreads) void bucket_sort_global_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    uint32_t vk) {
  bucket_sort_global_body(counts, caps, rstart, spill_off, spill_map, slots, cap_slots, offsets, RW, K, out, list, list_n, vk, blockIdx.x, gridDim.x);
}

// ---------------------------------- buckets above the LDS caps: MSD split --
// A bucket of more than kMidCap records is split, most significant varying
// composite byte first, into pieces that the small-bucket sort can finish:
//  * msd_split: one block per bucket.  Its entries {composite, slot} go to
//    buffer B and are scattered by the first varying byte into buffer A; a
//    piece still larger than kSegCap is pushed on the bucket's own stack and
//    later scattered by its own first varying byte into the other buffer,
//    depth first, until no piece is left.  Consecutive digits whose pieces fit
//    kSegCap together form one segment; a segment only needs sorting within
//    itself.
//  * seg_sort: each segment sorted in LDS as a small bucket; its slot numbers
//    go, in sorted order, to the bucket's reference list.
//  * big_gather: each bucket's records copied out in the order of its list.
// Everything lives in the bucket's own output range (R*n bytes, not written
// yet): A = [0, 20n), B = [20n, 40n), the stack = [40n, (R-4)n), the
// reference list = [(R-4)n, Rn), R >= 64.  A split of c entries pushes at most
// c / kSegCap pieces, so the stack holds at most 14 n / 2048 entries of 16
// bytes.  The gather reads list chunk k0.. before writing records k0.., and
// record k ends at byte R(k+1) <= (R-4)n + 4(k+1) only for k = n-1, inside
// its own chunk.
constexpr uint32_t kSegCap = kSmallCap;
constexpr uint32_t kMsdThreads = 1024;
constexpr uint32_t kMsdWaves = kMsdThreads / 64;
constexpr uint32_t kMsdUnroll = 4;  // entries a thread loads together in a scatter step

__device__ __forceinline__ uint32_t first_varying_byte(uint32_t vary) {  // vary != 0
  return (uint32_t)__builtin_ctz(vary);  // bit p = composite byte p, byte 0 most significant
}

struct MsdShared {
  uint32_t top, overflow;  // the bucket's piece stack
  uint4 seg;               // piece being split
  uint32_t hist[256];
  uint32_t base[256];
  uint32_t cursor[256];
  uint4 sh_or[kMsdWaves], sh_and[kMsdWaves];
  uint32_t sh_scan[kMsdWaves + 1];
};

// Scatter X[s, s+c) into Y[s, s+c) by composite byte p (digit order, any
// order within a digit) and record the pieces: runs of whole digits of at
// most kSegCap entries become segments, larger digits go to the next level.
__device__ void msd_scatter(MsdShared& sh, const uint32_t* __restrict__ X, uint32_t* __restrict__ Y, uint32_t j,
                            uint32_t s, uint32_t c, uint32_t p, uint32_t yflag, uint4* __restrict__ leaf,
                            uint32_t* __restrict__ leaf_n, uint32_t leaf_cap, uint32_t* __restrict__ stack,
                            uint32_t stack_cap) {
  const uint32_t tid = threadIdx.x;
  if (tid < 256) sh.hist[tid] = 0;
  __syncthreads();
  // kMsdUnroll entries a thread per step, their loads issued together before
  // any is used (past the end: the last entry again, not counted); with one
  // entry a step, every step had waited for its own load
  for (uint32_t i0 = 0; i0 < c; i0 += kMsdUnroll * kMsdThreads) {
    uint32_t dd[kMsdUnroll];
#pragma unroll
    for (uint32_t u = 0; u < kMsdUnroll; ++u) {
      const uint32_t i = i0 + u * kMsdThreads + tid;
      dd[u] = digit_of(get_key(X, s + (i < c ? i : c - 1)), p);
    }
#pragma unroll
    for (uint32_t u = 0; u < kMsdUnroll; ++u) {
      const uint32_t i = i0 + u * kMsdThreads + tid;
      const bool valid = i < c;
      const uint32_t d = valid ? dd[u] : 0u;
      const uint64_t peers = match_digit8(d, valid);
      if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&sh.hist[d], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  // exclusive scan of the 256 digit counts by the first four waves
  if (tid < 256) {
    const uint32_t v = sh.hist[tid];
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off);
      if (lane_id() >= (uint32_t)off) x += y;
    }
    if (lane_id() == 63) sh.sh_scan[tid >> 6] = x;
    sh.base[tid] = x - v;
  }
  __syncthreads();
  if (tid < 256) {
    uint32_t add = 0;
    for (uint32_t q = 0; q < (tid >> 6); ++q) add += sh.sh_scan[q];
    sh.base[tid] += add;
    sh.cursor[tid] = sh.base[tid];
  }
  __syncthreads();
  for (uint32_t i0 = 0; i0 < c; i0 += kMsdUnroll * kMsdThreads) {
    uint32_t e[kMsdUnroll][5];
#pragma unroll
    for (uint32_t u = 0; u < kMsdUnroll; ++u) {
      const uint32_t i = i0 + u * kMsdThreads + tid;
      const uint32_t* src = X + 5ull * (s + (i < c ? i : c - 1));
#pragma unroll
      for (uint32_t w = 0; w < 5; ++w) e[u][w] = src[w];
    }
#pragma unroll
    for (uint32_t u = 0; u < kMsdUnroll; ++u) {
      const uint32_t i = i0 + u * kMsdThreads + tid;
      const bool valid = i < c;
      const uint32_t d = valid ? digit_of(make_uint4(e[u][0], e[u][1], e[u][2], e[u][3]), p) : 0u;
      const uint64_t peers = match_digit8(d, valid);
      const uint32_t leader = peers ? (uint32_t)__builtin_ctzll(peers) : 0u;
      uint32_t got = 0;
      if (valid && lane_id() == leader) got = atomicAdd(&sh.cursor[d], (uint32_t)__popcll(peers));
      got = __shfl(got, (int)leader);
      if (valid) {
        uint32_t* dst = Y + 5ull * (s + got + (uint32_t)__popcll(peers & lanemask_lt()));
#pragma unroll
        for (uint32_t w = 0; w < 5; ++w) dst[w] = e[u][w];
      }
    }
  }
  __syncthreads();
  if (tid == 0) {  // pieces, in digit order
    uint32_t run_s = 0, run_c = 0;
    auto flush = [&]() {
      if (run_c) {
        const uint32_t q = atomicAdd(leaf_n, 1u);
        if (q < leaf_cap) leaf[q] = make_uint4(j, s + run_s, run_c, yflag);
      }
      run_c = 0;
    };
    for (uint32_t d = 0; d < 256; ++d) {
      const uint32_t cd = sh.hist[d], bd = sh.base[d];
      if (cd == 0) continue;
      if (cd > kSegCap) {  // pushed on the bucket's stack: {start, count, buffer}
        flush();
        const uint32_t q = sh.top;
        if (q < stack_cap) {
          stack[3 * q] = s + bd;
          stack[3 * q + 1] = cd;
          stack[3 * q + 2] = yflag;
          sh.top = q + 1;
        } else {
          sh.overflow = 1;
        }
        continue;
      }
      if (run_c + cd > kSegCap) flush();
      if (run_c == 0) run_s = bd;
      run_c += cd;
    }
    flush();
  }
  __syncthreads();
}

__device__ __forceinline__ void bucket_bufs(uint32_t* out, uint64_t out0, uint32_t n, uint32_t RW, uint32_t** A,
                                            uint32_t** B) {
  uint32_t* o_dw = out + out0 * RW;
  *A = o_dw;
  *B = o_dw + 5ull * n;
}

__device__ __forceinline__ void msd_split_body(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    uint4* __restrict__ leaf, uint32_t* __restrict__ leaf_n, uint32_t leaf_cap, uint32_t* __restrict__ error,
    uint32_t vk, uint32_t bid,
    uint32_t nblk) {
  __shared__ MsdShared sh;
  const uint32_t W = slot_bytes_for(RW * 4) / 4;
  const uint32_t nitems = *list_n;
  for (uint32_t it = bid; it < nitems; it += nblk) {
    const uint32_t j = list[it];
    BucketRef br;
    br.n = counts[j];
    const uint32_t cap = caps[j];
    br.nr = br.n < cap ? br.n : cap;
    br.rs = rstart[j];
    br.so = spill_off[j];
    br.out0 = offsets[j];
    uint32_t *A, *Bf;
    bucket_bufs(out, br.out0, br.n, RW, &A, &Bf);
    uint32_t* stack = out + br.out0 * RW + 10ull * br.n;                 // byte 40n
    const uint32_t stack_cap = (uint32_t)(((uint64_t)(RW - 11) * br.n) / 3);  // dwords [10n, (RW-1)n)
    if (threadIdx.x == 0) {
      sh.top = 0;
      sh.overflow = 0;
    }
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    // kMsdUnroll slot heads a thread per step, loaded together (past the end:
    // the last slot again, not stored)
    for (uint32_t q0 = 0; q0 < br.n; q0 += kMsdUnroll * kMsdThreads) {
      uint32_t sl[kMsdUnroll];
#pragma unroll
      for (uint32_t u = 0; u < kMsdUnroll; ++u) {
        const uint32_t q = q0 + u * kMsdThreads + threadIdx.x;
        sl[u] = slot_of(br, q < br.n ? q : br.n - 1, spill_map, cap_slots);
      }
      uint4 hv[kMsdUnroll];
#pragma unroll
      for (uint32_t u = 0; u < kMsdUnroll; ++u) hv[u] = *reinterpret_cast<const uint4*>(slots + (uint64_t)sl[u] * W);
#pragma unroll
      for (uint32_t u = 0; u < kMsdUnroll; ++u) {
        const uint32_t q = q0 + u * kMsdThreads + threadIdx.x;
        if (q < br.n) {
          uint32_t r0 = hv[u].y, r1 = hv[u].z, r2 = hv[u].w;
          virtual_key(r0, r1, r2, vk);
          const uint4 c = composite_words(hv[u].x, r0, r1, r2, K);
          put_entry(Bf, q, c, sl[u]);
          o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
          a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
        }
      }
    }
    uint32_t vary = varying_bytes<kMsdThreads>(o, a, sh.sh_or, sh.sh_and);  // syncs
    msd_scatter(sh, Bf, A, j, 0, br.n, first_varying_byte(vary), 0u, leaf, leaf_n, leaf_cap, stack, stack_cap);
    // depth first over the pieces still above kSegCap
    for (;;) {
      if (threadIdx.x == 0) {
        if (sh.top > 0) {
          const uint32_t q = --sh.top;
          sh.seg = make_uint4(stack[3 * q], stack[3 * q + 1], stack[3 * q + 2], 1u);
        } else {
          sh.seg = make_uint4(0, 0, 0, 0);
        }
      }
      __syncthreads();
      const uint4 sg = sh.seg;  // start, count, buffer, valid
      __syncthreads();
      if (!sg.w) break;
      const uint32_t* X = sg.z ? Bf : A;
      uint32_t* Y = sg.z ? A : Bf;
      o = make_uint4(0, 0, 0, 0);
      a = make_uint4(~0u, ~0u, ~0u, ~0u);
      for (uint32_t q0 = 0; q0 < sg.y; q0 += kMsdUnroll * kMsdThreads) {
        uint4 kv[kMsdUnroll];  // loaded together; past the piece's end its last entry again
#pragma unroll
        for (uint32_t u = 0; u < kMsdUnroll; ++u) {
          const uint32_t q = q0 + u * kMsdThreads + threadIdx.x;
          kv[u] = get_key(X, sg.x + (q < sg.y ? q : sg.y - 1));
        }
#pragma unroll
        for (uint32_t u = 0; u < kMsdUnroll; ++u) {
          const uint4 c = kv[u];  // a repeated entry changes neither the OR nor the AND
          o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
          a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
        }
      }
      vary = varying_bytes<kMsdThreads>(o, a, sh.sh_or, sh.sh_and);
      msd_scatter(sh, X, Y, j, sg.x, sg.y, first_varying_byte(vary), sg.z ^ 1u, leaf, leaf_n, leaf_cap, stack,
                  stack_cap);
    }
    if (threadIdx.x == 0 && sh.overflow) atomicOr(error, 1u);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kMsdThreads) void msd_split_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    uint4* __restrict__ leaf, uint32_t* __restrict__ leaf_n, uint32_t leaf_cap, uint32_t* __restrict__ error,
    uint32_t vk) {
  msd_split_body(counts, caps, rstart, spill_off, spill_map, slots, cap_slots, offsets, RW, K, out, list, list_n, leaf, leaf_n, leaf_cap, error, vk, blockIdx.x, gridDim.x);
}

// One segment per block: the small-bucket sort on entries from the buffer;
// the sorted slot numbers go to the bucket's reference list.
__device__ __forceinline__ void seg_sort_body(const uint32_t* __restrict__ counts,
                                                              const uint64_t* __restrict__ offsets, uint32_t RW,
                                                              uint32_t* __restrict__ out,
                                                              const uint4* __restrict__ segs,
                                                              const uint32_t* __restrict__ segs_n, uint32_t segs_cap, uint32_t bid,
    uint32_t nblk) {
  constexpr uint32_t AR = kSmCap / kSmThreads;
  __shared__ uint32_t cw[4][kSmCap];
  __shared__ uint16_t perm[2][kSmCap];
  __shared__ uint32_t bins[1u << kSmBits];
  __shared__ uint4 sh_or[kSmWaves], sh_and[kSmWaves];
  __shared__ uint32_t sh_scan[kSmThreads / 64 + 1];
  __shared__ uint64_t sh_mm[2 * kSmWaves];
  __shared__ uint32_t tot[4];
  const uint32_t tid = threadIdx.x;
  const uint32_t nseg = *segs_n < segs_cap ? *segs_n : segs_cap;
  for (uint32_t it = bid; it < nseg; it += nblk) {
    const uint4 sg = segs[it];
    const uint32_t nb = counts[sg.x], n = sg.z;
    uint32_t *A, *Bf;
    bucket_bufs(out, offsets[sg.x], nb, RW, &A, &Bf);
    const uint32_t* X = (sg.w ? Bf : A) + 5ull * sg.y;
    uint32_t* refs = out + offsets[sg.x] * RW + (uint64_t)(RW - 1) * nb + sg.y;
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    uint4 kv[AR];  // every key load in flight together (past the end: the last entry again)
#pragma unroll
    for (uint32_t i = 0; i < AR; ++i) {
      const uint32_t q = tid + i * kSmThreads;
      kv[i] = get_key(X, q < n ? q : n - 1);
    }
#pragma unroll
    for (uint32_t i = 0; i < AR; ++i) {
      const uint32_t q = tid + i * kSmThreads;
      if (q < n) {
        const uint4 c = kv[i];
        cw[0][q] = c.x; cw[1][q] = c.y; cw[2][q] = c.z; cw[3][q] = c.w;
        o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
        a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
      }
    }
    const uint32_t vary = vary_mask(block_diff<kSmThreads>(o, a, sh_or, sh_and));
    // the counting digit: the key's base-95 code scaled over its range in the
    // segment; when the code is the same for the whole segment (one key, or
    // keys equal in their first 8 bytes), the 8 composite bytes from the first
    // varying one (key bytes 8.. and the index) instead
    uint64_t cmin = ~0ull, cmax = 0;
    for (uint32_t q = tid; q < n; q += kSmThreads) {
      const uint64_t e = key_code(__builtin_bswap32(cw[0][q]), __builtin_bswap32(cw[1][q]));
      cmin = e < cmin ? e : cmin;
      cmax = e > cmax ? e : cmax;
    }
    block_min_max_u64<kSmThreads>(cmin, cmax, sh_mm);
    const bool by_code = cmax > cmin;
    const uint32_t p0 = vary ? (uint32_t)__builtin_ctz(vary) : 0u;
    auto digit_src = [&](uint32_t q) -> uint64_t {
      if (by_code) return key_code(__builtin_bswap32(cw[0][q]), __builtin_bswap32(cw[1][q]));
      const uint32_t wd = p0 >> 2, sh = 8 * (p0 & 3);
      const uint64_t hi = ((uint64_t)cw[wd][q] << 32) | (wd + 1 < 4 ? cw[wd + 1][q] : 0u);
      const uint32_t nx = wd + 2 < 4 ? cw[wd + 2][q] : 0u;
      return sh ? (hi << sh) | (nx >> (32 - sh)) : hi;
    };
    if (!by_code) {
      cmin = ~0ull;
      cmax = 0;
      for (uint32_t q = tid; q < n; q += kSmThreads) {
        const uint64_t wv = digit_src(q);
        cmin = wv < cmin ? wv : cmin;
        cmax = wv > cmax ? wv : cmax;
      }
      block_min_max_u64<kSmThreads>(cmin, cmax, sh_mm);
    }
    uint32_t cur = 0;
    if (n == 1) {
      if (tid == 0) perm[0][0] = 0;
    } else {
      const double scale = (double)(1u << kSmBits) / ((double)(cmax - cmin) + 1.0);
      for (uint32_t i = tid; i < (1u << kSmBits); i += kSmThreads) bins[i] = 0;
      for (uint32_t q = tid; q < n; q += kSmThreads) {
        const uint32_t d = (uint32_t)((double)(digit_src(q) - cmin) * scale);
        perm[1][q] = (uint16_t)(d < (1u << kSmBits) ? d : (1u << kSmBits) - 1);
      }
      cur = small_sort_core(n, vary, cw, perm, bins, sh_scan, tot, scaled_pos(digit_src, cmin, scale));
    }
    __syncthreads();
    for (uint32_t k = tid; k < n; k += kSmThreads) refs[k] = X[5ull * perm[cur][k] + 4];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSmThreads) void seg_sort_kernel(const uint32_t* __restrict__ counts,
                                                              const uint64_t* __restrict__ offsets, uint32_t RW,
                                                              uint32_t* __restrict__ out,
                                                              const uint4* __restrict__ segs,
                                                              const uint32_t* __restrict__ segs_n, uint32_t segs_cap) {
  seg_sort_body(counts, offsets, RW, out, segs, segs_n, segs_cap, blockIdx.x, gridDim.x);
}

// Each bucket's records in the order of its reference list: lane q moves
// 16-byte chunk q % LC of record q / LC (one slot line per record).
constexpr uint32_t kGatherChunk = 4096;

__device__ __forceinline__ void big_gather_body(const uint32_t* __restrict__ counts,
                                                                 const uint64_t* __restrict__ offsets, uint32_t RW,
                                                                 const uint4* __restrict__ slots,
                                                                 uint32_t* __restrict__ out,
                                                                 const uint32_t* __restrict__ list,
                                                                 const uint32_t* __restrict__ list_n, uint32_t bid,
    uint32_t nblk) {
  __shared__ uint32_t chunk_slot[kGatherChunk];
  const uint32_t SC = slot_bytes_for(RW * 4) / 16;
  const uint32_t LC = (RW + 1 + 3) / 4;
  const uint32_t nitems = *list_n;
  for (uint32_t it = bid; it < nitems; it += nblk) {
    const uint32_t j = list[it], n = counts[j];
    uint32_t* o_dw = out + offsets[j] * RW;
    const uint32_t* refs = o_dw + (uint64_t)(RW - 1) * n;
    for (uint32_t k0 = 0; k0 < n; k0 += kGatherChunk) {
      const uint32_t m = n - k0 < kGatherChunk ? n - k0 : kGatherChunk;
      for (uint32_t i = threadIdx.x; i < m; i += kMsdThreads) chunk_slot[i] = refs[k0 + i];
      __syncthreads();
      const uint32_t nq = m * LC;
      for (uint32_t q0 = 0; q0 < nq; q0 += kSmGroup * kMsdThreads) {
        u32x4 g[kSmGroup];
#pragma unroll
        for (uint32_t i = 0; i < kSmGroup; ++i) {  // kSmGroup loads in flight before the stores
          const uint32_t q = q0 + threadIdx.x + i * kMsdThreads;
          const uint32_t qq = q < nq ? q : nq - 1;
          const uint32_t k = qq / LC, c = qq - k * LC;
          g[i] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(slots) + (uint64_t)chunk_slot[k] * SC + c);
        }
#pragma unroll
        for (uint32_t i = 0; i < kSmGroup; ++i) {
          const uint32_t q = q0 + threadIdx.x + i * kMsdThreads;
          if (q < nq) {
            const uint32_t k = q / LC, c = q - k * LC;
            uint32_t* o = o_dw + (uint64_t)(k0 + k) * RW;
#pragma unroll
            for (uint32_t t = 0; t < 4; ++t) {
              const uint32_t sd = 4 * c + t;  // slot dword: 0 is the index, 1..RW the record
              if (sd >= 1 && sd <= RW) o[sd - 1] = g[i][t];
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kMsdThreads) void big_gather_kernel(const uint32_t* __restrict__ counts,
                                                                 const uint64_t* __restrict__ offsets, uint32_t RW,
                                                                 const uint4* __restrict__ slots,
                                                                 uint32_t* __restrict__ out,
                                                                 const uint32_t* __restrict__ list,
                                                                 const uint32_t* __restrict__ list_n) {
  big_gather_body(counts, offsets, RW, slots, out, list, list_n, blockIdx.x, gridDim.x);
}




// ------------------------------------------- whole jobs of up to 2048 records --
// A batch's small jobs need no partition: one block sorts a whole job the way
// the small-bucket kernel sorts a bucket, reading the keys straight from the
// job's records.  An in-place job is first copied to its staging area.
__global__ __launch_bounds__(kSmThreads) void tiny_jobs_kernel(const TinyJob* __restrict__ jobs, uint32_t njobs,
                                                               uint32_t RW, uint32_t K, uint32_t* __restrict__ staging) {
  constexpr uint32_t AR = kSmCap / kSmThreads;
  __shared__ uint32_t cw[4][kSmCap];
  __shared__ uint16_t perm[2][kSmCap];
  __shared__ uint32_t bins[1u << kSmBits];
  __shared__ uint4 sh_or[kSmWaves], sh_and[kSmWaves];
  __shared__ uint32_t sh_scan[kSmThreads / 64 + 1];
  __shared__ uint64_t sh_mm[2 * kSmWaves];
  __shared__ uint32_t tot[4];
  const uint32_t tid = threadIdx.x;
  for (uint32_t jb = blockIdx.x; jb < njobs; jb += gridDim.x) {
    const TinyJob J = jobs[jb];
    const uint32_t n = J.n;
    const uint32_t* src = J.in;
    if (J.in == J.out) {  // in place: keep a copy to gather from
      uint32_t* stg = staging + J.staging_dw;
      for (uint32_t f = tid; f < n * RW; f += kSmThreads) stg[f] = J.in[f];
      __syncthreads();
      src = stg;
    }
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    uint64_t cmin = ~0ull, cmax = 0;
    uint32_t kr[AR][3];  // every key load in flight together (past the end: the last record again)
#pragma unroll
    for (uint32_t i = 0; i < AR; ++i) {
      const uint32_t q = tid + i * kSmThreads;
      const uint32_t* r = src + (uint64_t)(q < n ? q : n - 1) * RW;
      kr[i][0] = r[0];
      kr[i][1] = r[1];
      kr[i][2] = r[2];
    }
#pragma unroll
    for (uint32_t i = 0; i < AR; ++i) {
      const uint32_t q = tid + i * kSmThreads;
      if (q < n) {
        const uint32_t* r = kr[i];
        const uint4 c = composite_words(q, r[0], r[1], r[2], K);
        cw[0][q] = c.x; cw[1][q] = c.y; cw[2][q] = c.z; cw[3][q] = c.w;
        o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
        a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
        const uint64_t e = key_code(r[0], r[1]);
        cmin = e < cmin ? e : cmin;
        cmax = e > cmax ? e : cmax;
      }
    }
    const uint4 diff = block_diff<kSmThreads>(o, a, sh_or, sh_and);
    const uint32_t vary = vary_mask(diff);
    block_min_max_u64<kSmThreads>(cmin, cmax, sh_mm);
    uint32_t cur = 0;
    if (n == 1) {
      if (tid == 0) perm[0][0] = 0;
    } else {
      const double scale = (double)(1u << kSmBits) / ((double)(cmax - cmin) + 1.0);
      for (uint32_t i = tid; i < (1u << kSmBits); i += kSmThreads) bins[i] = 0;
      for (uint32_t q = tid; q < n; q += kSmThreads) {
        const uint32_t* r = src + (uint64_t)q * RW;
        const uint64_t e = key_code(r[0], r[1]);
        const uint32_t d = (uint32_t)((double)(e - cmin) * scale);
        perm[1][q] = (uint16_t)(d < (1u << kSmBits) ? d : (1u << kSmBits) - 1);
      }
      auto code_of = [&](uint32_t q) -> uint64_t {
        const uint32_t* r = src + (uint64_t)q * RW;
        return key_code(r[0], r[1]);
      };
      cur = small_sort_core(n, vary, cw, perm, bins, sh_scan, tot, scaled_pos(code_of, cmin, scale));
    }
    __syncthreads();
    for (uint32_t f = tid; f < n * RW; f += kSmThreads) {
      const uint32_t k = f / RW, d = f - k * RW;
      J.out[f] = src[(uint64_t)perm[cur][k] * RW + d];
    }
    __syncthreads();
  }
}

hipError_t launch_tiny_jobs(const TinyJob* d_jobs, uint32_t njobs, uint32_t rec_bytes, uint32_t key_bytes,
                            uint32_t* staging, hipStream_t st) {
  if (njobs == 0) return hipSuccess;
  tiny_jobs_kernel<<<njobs < 4096 ? njobs : 4096, kSmThreads, 0, st>>>(d_jobs, njobs, rec_bytes / 4, key_bytes,
                                                                       staging);
  return hipGetLastError();
}

// ------------------------------------------- keys longer than 12 bytes --
// Section 4: key bytes past the encoded prefix are ordered by a last-mile
// step.  The bucket sorts order records by (key bytes 0..11, input index).  With a
// longer key, records whose first 12 key bytes agree therefore sit next to
// each other in input order, and each such run only needs a stable sort by
// key bytes 12..K-1.  Equal 12-byte prefixes have equal 8-byte codes, so a run
// never crosses a bucket.

__device__ __forceinline__ bool same_prefix12(const uint32_t* a, const uint32_t* b) {
  return a[0] == b[0] && a[1] == b[1] && a[2] == b[2];
}

// Key bytes 12..K-1 of a record as four big-endian words, zero past the key
// (the record is dword-aligned and at least K bytes long, so every dword
// read holds a key byte and lies inside the record).
__device__ __forceinline__ uint4 key_suffix(const uint32_t* rec, uint32_t K) {
  uint32_t w[4];
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t b0 = 12 + 4 * q;
    uint32_t v = b0 < K ? __builtin_bswap32(rec[3 + q]) : 0u;
    if (b0 < K && K < b0 + 4) v &= ~0u << (8 * (b0 + 4 - K));
    w[q] = v;
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

__device__ __forceinline__ bool suffix_less(const uint4& a, const uint4& b) {
  if (a.x != b.x) return a.x < b.x;
  if (a.y != b.y) return a.y < b.y;
  if (a.z != b.z) return a.z < b.z;
  return a.w < b.w;
}

// The first record of every run of two or more equal 12-byte prefixes.
__global__ __launch_bounds__(256) void long_runs_kernel(const uint32_t* __restrict__ out, uint64_t n, uint32_t RW,
                                                        uint32_t* __restrict__ list, uint32_t* __restrict__ list_n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i + 1 >= n) return;
  const uint32_t* r = out + i * RW;
  if (!same_prefix12(r, r + RW)) return;
  if (i > 0 && same_prefix12(r - RW, r)) return;
  list[atomicAdd(list_n, 1u)] = (uint32_t)i;
}

// One block per run: find its end, leave it if it is already in suffix order
// (duplicates of one key are), else sort {suffix, position} entries stably by
// the varying suffix bytes and rewrite the run's records from a staged copy.
// ea, eb: 20-byte entries of run positions [s, s+len); stage: records.
__global__ __launch_bounds__(kBigThreads) void long_run_sort_kernel(
    uint32_t* __restrict__ out, uint64_t n, uint32_t RW, uint32_t K, const uint32_t* __restrict__ list,
    const uint32_t* __restrict__ list_n, uint32_t* __restrict__ ea, uint32_t* __restrict__ eb,
    uint32_t* __restrict__ stage) {
  __shared__ LsdShared lsd;
  __shared__ uint4 sh_or[kBigWaves], sh_and[kBigWaves];
  __shared__ uint32_t sh_len, sh_unsorted;
  const uint32_t nruns = *list_n;
  for (uint32_t it = blockIdx.x; it < nruns; it += gridDim.x) {
    const uint64_t s = list[it];
    uint32_t* rs = out + s * RW;
    // 1. the run's length: the first later record with another prefix
    if (threadIdx.x == 0) sh_len = 0xFFFFFFFFu;
    __syncthreads();
    for (uint64_t c0 = s + 1;; c0 += kBigThreads) {
      const uint64_t i = c0 + threadIdx.x;
      if (i < n && !same_prefix12(rs, out + i * RW)) atomicMin(&sh_len, (uint32_t)(i - s));
      __syncthreads();
      const uint32_t found = sh_len;
      __syncthreads();
      if (found != 0xFFFFFFFFu || c0 + kBigThreads >= n) break;
    }
    const uint32_t len = sh_len != 0xFFFFFFFFu ? sh_len : (uint32_t)(n - s);
    // 2. already in order?
    if (threadIdx.x == 0) sh_unsorted = 0;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k + 1 < len; k += kBigThreads)
      if (suffix_less(key_suffix(rs + (uint64_t)(k + 1) * RW, K), key_suffix(rs + (uint64_t)k * RW, K)))
        sh_unsorted = 1;
    __syncthreads();
    const bool unsorted = sh_unsorted != 0;
    __syncthreads();
    if (!unsorted) continue;
    // 3. entries and the suffix bytes that vary
    uint32_t* A = ea + 5 * s;
    uint32_t* Bf = eb + 5 * s;
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint32_t k = threadIdx.x; k < len; k += kBigThreads) {
      const uint4 c = key_suffix(rs + (uint64_t)k * RW, K);
      put_entry(A, k, c, k);
      o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
      a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
    }
    const uint32_t vary = varying_bytes<kBigThreads>(o, a, sh_or, sh_and);  // syncs
    // 4. stable LSD over them: equal suffixes keep their (input) order
    const uint32_t* res = lsd_entries(A, Bf, len, vary, K - kSortKeyBytes, lsd);
    // 5. the run's records in suffix order, through the stage
    uint32_t* st = stage + s * RW;
    const uint64_t total = (uint64_t)len * RW;
    for (uint64_t f = threadIdx.x; f < total; f += kBigThreads) st[f] = rs[f];
    __syncthreads();
    for (uint64_t f = threadIdx.x; f < total; f += kBigThreads) {
      const uint64_t k = f / RW, d = f - k * RW;
      rs[f] = st[(uint64_t)res[5 * k + 4] * RW + d];
    }
    __syncthreads();
  }
}

static size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t long_key_scratch_bytes(uint64_t n, uint32_t rec_bytes) {
  return al256(4) + al256((n / 2 + 1) * 4) + 2 * al256((size_t)n * 20) + al256((size_t)n * rec_bytes);
}

hipError_t launch_long_key_fixup(uint8_t* out, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, uint8_t* scratch,
                                 hipStream_t st) {
  if (key_bytes <= kSortKeyBytes || n < 2) return hipSuccess;
  uint8_t* p = scratch;
  uint32_t* list_n = reinterpret_cast<uint32_t*>(p);
  p += al256(4);
  uint32_t* list = reinterpret_cast<uint32_t*>(p);
  p += al256((n / 2 + 1) * 4);
  uint32_t* ea = reinterpret_cast<uint32_t*>(p);
  p += al256((size_t)n * 20);
  uint32_t* eb = reinterpret_cast<uint32_t*>(p);
  p += al256((size_t)n * 20);
  uint32_t* stage = reinterpret_cast<uint32_t*>(p);
  hipError_t err = launch_fill_u32(list_n, 1, 0u, st);
  if (err != hipSuccess) return err;
  const uint32_t RW = rec_bytes / 4;
  uint32_t* o = reinterpret_cast<uint32_t*>(out);
  long_runs_kernel<<<(uint32_t)((n + 255) / 256), 256, 0, st>>>(o, n, RW, list, list_n);
  long_run_sort_kernel<<<256, kBigThreads, 0, st>>>(o, n, RW, key_bytes, list, list_n, ea, eb, stage);
  return hipGetLastError();
}

struct SortArgs {
  const uint32_t *counts, *caps, *rstart, *soff, *smap, *slots;
  const PartHeader* ph;
  uint32_t* out;
  uint32_t RW;
};

static SortArgs sort_args(const uint8_t* part, const PartLayout& lay, uint32_t rec_bytes, uint8_t* out) {
  SortArgs a;
  a.counts = reinterpret_cast<const uint32_t*>(part + lay.counts);
  a.caps = reinterpret_cast<const uint32_t*>(part + lay.caps);
  a.rstart = reinterpret_cast<const uint32_t*>(part + lay.rstart);
  a.soff = reinterpret_cast<const uint32_t*>(part + lay.spill_off);
  a.smap = reinterpret_cast<const uint32_t*>(part + lay.spill_map);
  a.slots = reinterpret_cast<const uint32_t*>(part + lay.slots);
  a.ph = reinterpret_cast<const PartHeader*>(part + lay.header);
  a.out = reinterpret_cast<uint32_t*>(out);
  a.RW = rec_bytes / 4;
  return a;
}

hipError_t launch_bucket_sort_small(uint8_t* part, const PartLayout& lay, uint32_t B, const uint64_t* offsets,
                                    uint32_t rec_bytes, uint32_t key_bytes, uint8_t* out, hipStream_t st,
                                    uint32_t vk) {
  SortArgs a = sort_args(part, lay, rec_bytes, out);
  if (rec_bytes == 100) {
    bucket_sort_small_kernel<25><<<B, kSmThreads, 0, st>>>(a.counts, a.caps, a.rstart, a.soff, a.smap,
                                                           reinterpret_cast<const uint4*>(a.slots), lay.cap_slots,
                                                           offsets, key_bytes, a.out, B, vk);
  } else {
    bucket_sort_lds_kernel<kSmallCap, 256><<<B, 256, 0, st>>>(a.counts, a.caps, a.rstart, a.soff, a.smap, a.slots,
                                                               lay.cap_slots, offsets, a.RW, key_bytes, a.out,
                                                               nullptr, nullptr, false, B, nullptr, vk);
  }
  return hipGetLastError();
}

// The kernels below walk device-side lists with persistent blocks; their grids
// are sized from what n records can hold (at most n / 2049 mid buckets, n /
// 6145 big ones, about n / 1024 segments), so that the small jobs of a batch
// do not dispatch thousands of blocks that find nothing to do.
static uint32_t grid_for(uint64_t n, uint64_t per_block, uint32_t most) {
  const uint64_t g = n / per_block + 1;
  return (uint32_t)(g < most ? g : most);
}

hipError_t launch_bucket_sort_large(uint8_t* part, const PartLayout& lay, uint32_t B, uint64_t n,
                                    const uint64_t* offsets, uint32_t rec_bytes, uint32_t key_bytes, uint8_t* out,
                                    hipStream_t st, uint32_t vk) {
  SortArgs a = sort_args(part, lay, rec_bytes, out);
  PartHeader* ph = reinterpret_cast<PartHeader*>(part + lay.header);
  const uint32_t* mid_list = reinterpret_cast<const uint32_t*>(part + lay.mid_list);
  bucket_sort_lds_kernel<kMidLoCap, kMidLoThreads><<<grid_for(n, kSmallCap + 1, 512), kMidLoThreads, 0, st>>>(
      a.counts, a.caps, a.rstart, a.soff, a.smap, a.slots, lay.cap_slots, offsets, a.RW, key_bytes, a.out,
      mid_list, &ph->n_mid, false, B, ph, vk);
  bucket_sort_lds_kernel<kMidCap, kMidThreads><<<grid_for(n, kMidLoCap + 1, 256), kMidThreads, 0, st>>>(
      a.counts, a.caps, a.rstart, a.soff, a.smap, a.slots, lay.cap_slots, offsets, a.RW, key_bytes, a.out,
      mid_list, &ph->n_mid_hi, true, B, nullptr, vk);
  // buckets of one repeated key first; the others go on to big2
  uint32_t* big2 = reinterpret_cast<uint32_t*>(part + lay.big2_list);
  equal_keys_kernel<<<grid_for(n, kMidCap + 1, 256), kEqThreads, 0, st>>>(
      a.counts, a.caps, a.rstart, a.soff, a.smap, a.slots, lay.cap_slots, offsets, a.RW, key_bytes, a.out,
      reinterpret_cast<const uint32_t*>(part + lay.big_list), &a.ph->n_big, big2, &ph->n_big2, vk);
  if (rec_bytes < 64) {  // too little room for the split's buffers, stack and reference list
    bucket_sort_global_kernel<<<grid_for(n, kMidCap + 1, 256), kBigThreads, 0, st>>>(
        a.counts, a.caps, a.rstart, a.soff, a.smap, a.slots, lay.cap_slots, offsets, a.RW, key_bytes, a.out,
        big2, &ph->n_big2, vk);
    return hipGetLastError();
  }
  uint4* leaf = reinterpret_cast<uint4*>(part + lay.seg_leaf);
  uint32_t* leaf_n = &ph->seg_n[0];
  const uint32_t leaf_cap = lay.seg_leaf_cap;
  // the split's counters (ph->seg_n) were cleared by the mid-bucket kernel
  msd_split_kernel<<<grid_for(n, kMidCap + 1, 512), kMsdThreads, 0, st>>>(
      a.counts, a.caps, a.rstart, a.soff, a.smap, a.slots, lay.cap_slots, offsets, a.RW, key_bytes, a.out, big2,
      &ph->n_big2, leaf, leaf_n, leaf_cap, &ph->seg_n[1], vk);
  seg_sort_kernel<<<grid_for(n, 1024, 2048), kSmThreads, 0, st>>>(a.counts, offsets, a.RW, a.out, leaf, leaf_n,
                                                                   leaf_cap);
  big_gather_kernel<<<grid_for(n, kMidCap + 1, 512), kMsdThreads, 0, st>>>(
      a.counts, offsets, a.RW, reinterpret_cast<const uint4*>(a.slots), a.out, big2, &ph->n_big2);
  return hipGetLastError();
}

// ---------------------------------------------------------- batch windows --
// The bucket sorts of a window of a batch: G blocks per job, block b working
// for job b / G as its block b % G of G.  Each kernel body is the one the
// single-job launches above run.
WinGrids window_grids(uint64_t nmax, uint32_t Bmax, uint32_t tiles_per_block) {
  WinGrids g;
  const uint64_t ntiles = (nmax + 255) / 256;  // partition tiles of the largest job
  g.part = tiles_per_block ? (uint32_t)std::min<uint64_t>((ntiles + tiles_per_block - 1) / tiles_per_block, 1u << 16)
                           : partition_grid(nmax);
  // Per job, the kernels after the small-bucket sort loop over their lists
  // with fewer blocks than one job of its size gets: a window launches them
  // for all its jobs at once, so the GPU stays full, and the empty blocks of
  // jobs with short lists (most of them) cost dispatch time
  g.fixup = std::min<uint32_t>(spill_fixup_grid(nmax), 256);
  g.small = Bmax;
  g.mid = grid_for(nmax, kSmallCap + 1, 64);
  g.split = grid_for(nmax, kMidCap + 1, 128);
  g.seg = grid_for(nmax, 1024, 256);
  g.gather = grid_for(nmax, kMidCap + 1, 128);
  return g;
}

struct WinRefs {  // a job's partition buffer as the bucket sorts read it
  const uint32_t *counts, *caps, *rstart, *soff, *smap, *slots;
  PartHeader* ph;
};

__device__ __forceinline__ WinRefs win_refs(const WinJob& J) {
  uint8_t* p = J.part;
  WinRefs r;
  r.counts = reinterpret_cast<const uint32_t*>(p + J.lay.counts);
  r.caps = reinterpret_cast<const uint32_t*>(p + J.lay.caps);
  r.rstart = reinterpret_cast<const uint32_t*>(p + J.lay.rstart);
  r.soff = reinterpret_cast<const uint32_t*>(p + J.lay.spill_off);
  r.smap = reinterpret_cast<const uint32_t*>(p + J.lay.spill_map);
  r.slots = reinterpret_cast<const uint32_t*>(p + J.lay.slots);
  r.ph = reinterpret_cast<PartHeader*>(p + J.lay.header);
  return r;
}

template <uint32_t RW>
__global__ __launch_bounds__(kSmThreads) void bucket_sort_small_win_kernel(const WinJob* __restrict__ jobs,
                                                                           uint32_t G, uint32_t K) {
  const WinJob& J = jobs[blockIdx.x / G];
  const WinRefs r = win_refs(J);
  bucket_sort_small_body<RW>(r.counts, r.caps, r.rstart, r.soff, r.smap, reinterpret_cast<const uint4*>(r.slots),
                             J.lay.cap_slots, J.offsets, K, reinterpret_cast<uint32_t*>(J.out), J.B, 0u,
                             blockIdx.x % G, G);
}

// MID 1: the mid list's buckets of up to kMidLoCap records (from its start;
// this first kernel of the chain also clears the split's counters); MID 2:
// its larger ones (from its end); MID 0: every bucket up to kSmallCap records
// (records other than 100 bytes).
template <uint32_t CAP, uint32_t THREADS, int MID>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(CAP == kMidLoCap ? 4 : 1))) void bucket_sort_lds_win_kernel(const WinJob* __restrict__ jobs, uint32_t G,
                                                                      uint32_t RW, uint32_t K) {
  const WinJob& J = jobs[blockIdx.x / G];
  const WinRefs r = win_refs(J);
  bucket_sort_lds_body<CAP, THREADS>(r.counts, r.caps, r.rstart, r.soff, r.smap, r.slots, J.lay.cap_slots, J.offsets,
                                     RW, K, reinterpret_cast<uint32_t*>(J.out),
                                     MID ? reinterpret_cast<const uint32_t*>(J.part + J.lay.mid_list) : nullptr,
                                     MID == 1 ? &r.ph->n_mid : (MID == 2 ? &r.ph->n_mid_hi : nullptr), MID == 2,
                                     J.B, MID == 1 ? r.ph : nullptr, 0u, blockIdx.x % G, G);
}

__global__ __launch_bounds__(kEqThreads) void equal_keys_win_kernel(const WinJob* __restrict__ jobs, uint32_t G,
                                                                    uint32_t RW, uint32_t K) {
  const WinJob& J = jobs[blockIdx.x / G];
  const WinRefs r = win_refs(J);
  equal_keys_body(r.counts, r.caps, r.rstart, r.soff, r.smap, r.slots, J.lay.cap_slots, J.offsets, RW, K,
                  reinterpret_cast<uint32_t*>(J.out), reinterpret_cast<const uint32_t*>(J.part + J.lay.big_list),
                  &r.ph->n_big, reinterpret_cast<uint32_t*>(J.part + J.lay.big2_list), &r.ph->n_big2, 0u,
                  blockIdx.x % G, G);
}

__global__ __launch_bounds__(kBigThreads) void bucket_sort_global_win_kernel(const WinJob* __restrict__ jobs,
                                                                             uint32_t G, uint32_t RW, uint32_t K) {
  const WinJob& J = jobs[blockIdx.x / G];
  const WinRefs r = win_refs(J);
  bucket_sort_global_body(r.counts, r.caps, r.rstart, r.soff, r.smap, r.slots, J.lay.cap_slots, J.offsets, RW, K,
                          reinterpret_cast<uint32_t*>(J.out), reinterpret_cast<const uint32_t*>(J.part + J.lay.big2_list),
                          &r.ph->n_big2, 0u, blockIdx.x % G, G);
}

__global__ __launch_bounds__(kMsdThreads) void msd_split_win_kernel(const WinJob* __restrict__ jobs, uint32_t G,
                                                                    uint32_t RW, uint32_t K) {
  const WinJob& J = jobs[blockIdx.x / G];
  const WinRefs r = win_refs(J);
  msd_split_body(r.counts, r.caps, r.rstart, r.soff, r.smap, r.slots, J.lay.cap_slots, J.offsets, RW, K,
                 reinterpret_cast<uint32_t*>(J.out), reinterpret_cast<const uint32_t*>(J.part + J.lay.big2_list),
                 &r.ph->n_big2, reinterpret_cast<uint4*>(J.part + J.lay.seg_leaf), &r.ph->seg_n[0], J.lay.seg_leaf_cap,
                 &r.ph->seg_n[1], 0u, blockIdx.x % G, G);
}

__global__ __launch_bounds__(kSmThreads) void seg_sort_win_kernel(const WinJob* __restrict__ jobs, uint32_t G,
                                                                  uint32_t RW) {
  const WinJob& J = jobs[blockIdx.x / G];
  const WinRefs r = win_refs(J);
  seg_sort_body(r.counts, J.offsets, RW, reinterpret_cast<uint32_t*>(J.out),
                reinterpret_cast<const uint4*>(J.part + J.lay.seg_leaf), &r.ph->seg_n[0], J.lay.seg_leaf_cap,
                blockIdx.x % G, G);
}

__global__ __launch_bounds__(kMsdThreads) void big_gather_win_kernel(const WinJob* __restrict__ jobs, uint32_t G,
                                                                     uint32_t RW) {
  const WinJob& J = jobs[blockIdx.x / G];
  const WinRefs r = win_refs(J);
  big_gather_body(r.counts, J.offsets, RW, reinterpret_cast<const uint4*>(r.slots), reinterpret_cast<uint32_t*>(J.out),
                  reinterpret_cast<const uint32_t*>(J.part + J.lay.big2_list), &r.ph->n_big2, blockIdx.x % G, G);
}

hipError_t launch_bucket_sort_small_win(const WinJob* jobs, uint32_t njobs, uint32_t G, uint32_t rec_bytes,
                                        uint32_t key_bytes, hipStream_t st) {
  if (njobs == 0 || G == 0) return hipSuccess;
  if (rec_bytes == 100)
    bucket_sort_small_win_kernel<25><<<njobs * G, kSmThreads, 0, st>>>(jobs, G, key_bytes);
  else
    bucket_sort_lds_win_kernel<kSmallCap, 256, 0><<<njobs * G, 256, 0, st>>>(jobs, G, rec_bytes / 4, key_bytes);
  return hipGetLastError();
}

hipError_t launch_bucket_sort_large_win(const WinJob* jobs, uint32_t njobs, const WinGrids& g, uint32_t rec_bytes,
                                        uint32_t key_bytes, hipStream_t st) {
  if (njobs == 0) return hipSuccess;
  const uint32_t RW = rec_bytes / 4;
  bucket_sort_lds_win_kernel<kMidLoCap, kMidLoThreads, 1><<<njobs * g.mid, kMidLoThreads, 0, st>>>(jobs, g.mid, RW,
                                                                                                 key_bytes);
  bucket_sort_lds_win_kernel<kMidCap, kMidThreads, 2><<<njobs * g.mid, kMidThreads, 0, st>>>(jobs, g.mid, RW, key_bytes);
  // buckets of one repeated key first (as many blocks per job as the mid sort)
  equal_keys_win_kernel<<<njobs * g.mid, kEqThreads, 0, st>>>(jobs, g.mid, RW, key_bytes);
  if (rec_bytes < 64) {  // too little room for the split's buffers, stack and reference list
    const uint32_t G = g.split < 256 ? g.split : 256;
    bucket_sort_global_win_kernel<<<njobs * G, kBigThreads, 0, st>>>(jobs, G, RW, key_bytes);
    return hipGetLastError();
  }
  // the split's counters (seg_n) were cleared by the mid-bucket kernel
  msd_split_win_kernel<<<njobs * g.split, kMsdThreads, 0, st>>>(jobs, g.split, RW, key_bytes);
  seg_sort_win_kernel<<<njobs * g.seg, kSmThreads, 0, st>>>(jobs, g.seg, RW);
  big_gather_win_kernel<<<njobs * g.gather, kMsdThreads, 0, st>>>(jobs, g.gather, RW);
  return hipGetLastError();
}

}  // namespace elsar
