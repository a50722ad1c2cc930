// In-bucket sort and concatenation (gfx950): Section 3.4 (sort each partition)
// and Section 3.5 (write it at the exclusive prefix sum of the partition sizes,
// coalescing the records in sorted order).
//
// A bucket's records sit in its region (and possibly the spill area) as
// 128-byte slots: record, 32-bit input index, padding.  Each record gives a
// composite sort key: the key bytes and then the index, big-endian, so the
// composite order is the key's memcmp order with ties broken by input
// position, and all composites of a bucket differ.  Sorting uses stable LSD
// radix passes with 8-bit digits over composite bytes; a byte that is equal
// across the whole bucket needs no pass (an all-equal-key bucket only sorts
// its index bytes -- early termination on duplicates).
//
//  * bucket_sort_small: buckets of up to 2048 records, one 512-thread block
//    each.  The first 16 bytes of every slot (index and key) go to LDS; one
//    counting pass on the key's base-95 code scaled over the bucket's code
//    range into 2048 bins, then an insertion sort by the whole composite
//    inside each bin (a full LSD sort if a bin is long), orders them.  The records are then gathered in
//    sorted order, each slot read once, straight into the output.
//  * bucket_sort_lds: buckets of up to 6144 records (all varying composite
//    bytes, entries and permutation in LDS, records gathered from the slots).
//  * bucket_sort_global: larger buckets, one block each; the ping-pong entry
//    buffers live in the bucket's own output range, which holds R*n bytes and
//    is not written yet (R >= 40 leaves room for 2 * 20n bytes).
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

__device__ __forceinline__ uint4 composite(const uint32_t* __restrict__ s, uint32_t /*RW*/, uint32_t K) {
  return composite_words(s[0], s[1], s[2], s[3], K);
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
constexpr uint32_t kRunMax = 32;     // longest bin sorted by insertion

template <uint32_t RW>  // record dwords
__global__ __launch_bounds__(kSmThreads) void bucket_sort_small_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map, const uint4* __restrict__ slots,
    uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t K, uint32_t* __restrict__ out, uint32_t B) {
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
  const uint32_t j = blockIdx.x;
  if (j >= B) return;
  BucketRef br;
  br.n = counts[j];
  if (br.n == 0 || br.n > kSmCap) return;
  const uint32_t cap = caps[j];
  br.nr = br.n < cap ? br.n : cap;
  br.rs = rstart[j];
  br.so = spill_off[j];
  br.out0 = offsets[j];
  const uint32_t n = br.n;

  // 1. the first 16 bytes of every slot: index and key
  uint4 v[AR];
#pragma unroll
  for (uint32_t i = 0; i < AR; ++i) {
    uint32_t p = tid + i * kSmThreads;
    if (p < n) v[i] = slots[(uint64_t)slot_of(br, p, spill_map, cap_slots) * SC];
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
  auto less = [&](uint32_t x, uint32_t y) -> bool {
    if (cw[0][x] != cw[0][y]) return cw[0][x] < cw[0][y];
    if (cw[1][x] != cw[1][y]) return cw[1][x] < cw[1][y];
    if (cw[2][x] != cw[2][y]) return cw[2][x] < cw[2][y];
    return cw[3][x] < cw[3][y];
  };
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
    __syncthreads();
    for (uint32_t p = tid; p < n; p += kSmThreads) atomicAdd(&bins[dig[p]], 1u);
    __syncthreads();
    {  // exclusive scan of the bins: PER contiguous per thread
      constexpr uint32_t PER = (1u << kSmBits) / kSmThreads;
      uint32_t c[PER], sum = 0;
#pragma unroll
      for (uint32_t i = 0; i < PER; ++i) { c[i] = bins[tid * PER + i]; sum += c[i]; }
      uint32_t total;
      uint32_t run = block_exclusive_scan<uint32_t, kSmThreads>(sum, sh_scan, &total);
#pragma unroll
      for (uint32_t i = 0; i < PER; ++i) { bins[tid * PER + i] = run; run += c[i]; }
    }
    __syncthreads();
    for (uint32_t p = tid; p < n; p += kSmThreads) perm[0][atomicAdd(&bins[dig[p]], 1u)] = (uint16_t)p;
    __syncthreads();
    // bins[b] is now the end of bin b; the start is the end of bin b-1
    bool long_bin = false;
    for (uint32_t b = tid; b < (1u << kSmBits); b += kSmThreads) {
      uint32_t s0 = b ? bins[b - 1] : 0u, s1 = bins[b];
      if (s1 - s0 < 2) continue;
      if (s1 - s0 > kRunMax) { long_bin = true; continue; }
      for (uint32_t x = s0 + 1; x < s1; ++x) {  // insertion sort by the whole composite
        uint16_t e = perm[0][x];
        uint32_t y = x;
        while (y > s0 && less(e, perm[0][y - 1])) {
          perm[0][y] = perm[0][y - 1];
          --y;
        }
        perm[0][y] = e;
      }
    }
    long_bin = __syncthreads_or(long_bin);
    if (long_bin) {  // stable LSD over every varying composite byte
      auto wc = reinterpret_cast<uint32_t(*)[256]>(bins);
      for (int pb = 15; pb >= 0; --pb) {
        if (!((vary >> pb) & 1u)) continue;
        lsd_pass<kSmCap, kSmThreads>(perm, cur, n, wc, tot, [&](uint32_t e) {
          return (cw[pb >> 2][e] >> (24 - 8 * (pb & 3))) & 0xFFu;
        });
        cur ^= 1;
      }
    }
  }
  __syncthreads();
  // 3. gather the records in sorted order straight into the output: lane q
  //    moves 16-byte chunk q % LC of the record at sorted position q / LC, so
  //    the lanes of a wave cover a contiguous stretch of the output.  Loads go
  //    out kSmGroup per thread before any store waits on them.
  uint32_t* o_dw = out + br.out0 * RW;
  const uint32_t nq = n * LC;
  for (uint32_t q0 = 0; q0 < nq; q0 += kSmGroup * kSmThreads) {
    u32x4 g[kSmGroup];
#pragma unroll
    for (uint32_t i = 0; i < kSmGroup; ++i) {
      uint32_t q = q0 + tid + i * kSmThreads;
      uint32_t qq = q < nq ? q : nq - 1;  // clamped: no branch around the loads
      uint32_t k = qq / LC, c = qq - k * LC;
      g[i] = reinterpret_cast<const u32x4*>(slots)[(uint64_t)slot_of(br, perm[cur][k], spill_map, cap_slots) * SC + c];
    }
#pragma unroll
    for (uint32_t i = 0; i < kSmGroup; ++i) {
      uint32_t q = q0 + tid + i * kSmThreads;
      if (q < nq) {
        uint32_t k = q / LC, c = q - k * LC;
        uint32_t* o = o_dw + k * RW;
#pragma unroll
        for (uint32_t t = 0; t < 4; ++t) {
          uint32_t sd = 4 * c + t;  // slot dword: 0 is the index, 1..RW the record
          if (sd >= 1 && sd <= RW) o[sd - 1] = g[i][t];
        }
      }
    }
  }
}

// ------------------------------------------- buckets of up to 6144 records --
template <uint32_t CAP, uint32_t THREADS>
__global__ __launch_bounds__(THREADS) void bucket_sort_lds_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    uint32_t B) {
  constexpr uint32_t WAVES = THREADS / 64;
  static_assert(CAP % THREADS == 0, "cap is whole rounds");
  __shared__ uint4 ent[CAP];
  __shared__ uint16_t perm[2][CAP];
  __shared__ uint32_t wc[WAVES][256];
  __shared__ uint4 sh_or[WAVES], sh_and[WAVES];
  __shared__ uint32_t tot[4];
  const uint32_t W = slot_bytes_for(RW * 4) / 4;  // slot stride in dwords
  const uint32_t nitems = list ? *list_n : B;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const uint32_t j = list ? list[it] : it;
    BucketRef br;
    br.n = counts[j];
    if (br.n == 0 || br.n > CAP) continue;
    const uint32_t cap = caps[j];
    br.nr = br.n < cap ? br.n : cap;
    br.rs = rstart[j];
    br.so = spill_off[j];
    br.out0 = offsets[j];
    // 1. load the entries
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint32_t p = threadIdx.x; p < br.n; p += THREADS) {
      uint32_t sl = slot_of(br, p, spill_map, cap_slots);
      uint4 c = composite(slots + (uint64_t)sl * W, RW, K);
      ent[p] = c;
      perm[0][p] = (uint16_t)p;
      o.x |= c.x; o.y |= c.y; o.z |= c.z; o.w |= c.w;
      a.x &= c.x; a.y &= c.y; a.z &= c.z; a.w &= c.w;
    }
    uint32_t vary = varying_bytes<THREADS>(o, a, sh_or, sh_and);  // syncs
    // 2. LSD passes, least significant composite byte first
    uint32_t cur = 0;
    const uint32_t nb = K + 4;
    for (int pbyte = (int)nb - 1; pbyte >= 0; --pbyte) {
      if (!((vary >> pbyte) & 1u)) continue;
      lsd_pass<CAP, THREADS>(perm, cur, br.n, wc, tot,
                             [&](uint32_t e) { return digit_of(ent[e], (uint32_t)pbyte); });
      cur ^= 1;
    }
    // 3. copy records in sorted order to the output
    const uint32_t total = br.n * RW;
    uint32_t* o_dw = out + br.out0 * RW;
    for (uint32_t f = threadIdx.x; f < total; f += THREADS) {
      uint32_t k = f / RW, d = f - k * RW;
      uint32_t sl = slot_of(br, perm[cur][k], spill_map, cap_slots);
      o_dw[f] = slots[(uint64_t)sl * W + d + 1];
    }
    __syncthreads();
  }
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

__global__ __launch_bounds__(kBigThreads) void bucket_sort_global_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n) {
  __shared__ uint32_t wc[kBigWaves][256];
  __shared__ uint32_t run[256];
  __shared__ uint32_t hist[256];
  __shared__ uint4 sh_or[kBigWaves], sh_and[kBigWaves];
  __shared__ uint32_t tot[4];
  __shared__ uint32_t chunk_slot[kBigTile];
  const uint32_t W = slot_bytes_for(RW * 4) / 4;  // slot stride in dwords
  const uint32_t w = threadIdx.x >> 6;
  const uint32_t nitems = *list_n;
  for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
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
      uint4 c = composite(slots + (uint64_t)slot_of(br, p, spill_map, cap_slots) * W, RW, K);
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
      put_entry(cur, p, composite(slots + (uint64_t)sl * W, RW, K), sl);
    }
    __syncthreads();
    // 2. stable LSD passes through global memory
    for (int pbyte = (int)nb - 1; pbyte >= 0; --pbyte) {
      if (!((vary >> pbyte) & 1u)) continue;
      if (threadIdx.x < 256) hist[threadIdx.x] = 0;
      __syncthreads();
      for (uint32_t p = threadIdx.x; p < br.n; p += kBigThreads) atomicAdd(&hist[digit_of(get_key(cur, p), pbyte)], 1u);
      __syncthreads();
      if (threadIdx.x < 256) {  // exclusive scan of hist -> run
        uint32_t v = hist[threadIdx.x], x = v;
        for (int off = 1; off < 64; off <<= 1) {
          uint32_t y = __shfl_up(x, off);
          if (lane_id() >= (uint32_t)off) x += y;
        }
        if (lane_id() == 63) tot[threadIdx.x >> 6] = x;
        __syncthreads();
        uint32_t add = 0;
        for (uint32_t i = 0; i < (threadIdx.x >> 6); ++i) add += tot[i];
        run[threadIdx.x] = x - v + add;
      } else {
        __syncthreads();
      }
      __syncthreads();
      for (uint32_t t0 = 0; t0 < br.n; t0 += kBigTile) {
        for (uint32_t i = threadIdx.x; i < kBigWaves * 256; i += kBigThreads) (&wc[0][0])[i] = 0;
        __syncthreads();
        uint32_t dg[kBigRounds], lc[kBigRounds];
#pragma unroll
        for (uint32_t r = 0; r < kBigRounds; ++r) {
          uint32_t i = t0 + w * (kBigRounds * 64) + r * 64 + lane_id();
          bool valid = i < br.n;
          uint32_t d = valid ? digit_of(get_key(cur, i), pbyte) : 0u;
          uint64_t peers = match_digit8(d, valid);
          uint32_t rank = __popcll(peers & lanemask_lt());
          uint32_t prev = valid ? wc[w][d] : 0u;
          __builtin_amdgcn_wave_barrier();
          if (valid && rank == 0) wc[w][d] = prev + (uint32_t)__popcll(peers);
          __builtin_amdgcn_wave_barrier();
          dg[r] = d;
          lc[r] = prev + rank;
        }
        __syncthreads();
        // per digit: tile count and wave offsets; then global position = run + offset
        if (threadIdx.x < 256) {
          uint32_t d = threadIdx.x, s = 0;
          for (uint32_t ww = 0; ww < kBigWaves; ++ww) {
            uint32_t c = wc[ww][d];
            wc[ww][d] = s + run[d];
            s += c;
          }
          hist[d] = s;  // this tile's count of digit d
        }
        __syncthreads();
#pragma unroll
        for (uint32_t r = 0; r < kBigRounds; ++r) {
          uint32_t i = t0 + w * (kBigRounds * 64) + r * 64 + lane_id();
          if (i < br.n) {
            const uint32_t* src = cur + 5ull * i;
            uint32_t dpos = wc[w][dg[r]] + lc[r];
            uint32_t* dst = nxt + 5ull * dpos;
            dst[0] = src[0]; dst[1] = src[1]; dst[2] = src[2]; dst[3] = src[3]; dst[4] = src[4];
          }
        }
        __syncthreads();
        if (threadIdx.x < 256) run[threadIdx.x] += hist[threadIdx.x];
        __syncthreads();
      }
      uint32_t* t = cur;
      cur = nxt;
      nxt = t;
    }
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

hipError_t launch_bucket_sort_small(const uint8_t* part, const PartLayout& lay, uint32_t B, const uint64_t* offsets,
                                    uint32_t rec_bytes, uint32_t key_bytes, uint8_t* out, hipStream_t st) {
  SortArgs a = sort_args(part, lay, rec_bytes, out);
  if (rec_bytes == 100) {
    bucket_sort_small_kernel<25><<<B, kSmThreads, 0, st>>>(a.counts, a.caps, a.rstart, a.soff, a.smap,
                                                           reinterpret_cast<const uint4*>(a.slots), lay.cap_slots,
                                                           offsets, key_bytes, a.out, B);
  } else {
    bucket_sort_lds_kernel<kSmallCap, 256><<<B, 256, 0, st>>>(a.counts, a.caps, a.rstart, a.soff, a.smap, a.slots,
                                                               lay.cap_slots, offsets, a.RW, key_bytes, a.out,
                                                               nullptr, nullptr, B);
  }
  return hipGetLastError();
}

hipError_t launch_bucket_sort_large(const uint8_t* part, const PartLayout& lay, uint32_t B, const uint64_t* offsets,
                                    uint32_t rec_bytes, uint32_t key_bytes, uint8_t* out, hipStream_t st) {
  SortArgs a = sort_args(part, lay, rec_bytes, out);
  bucket_sort_lds_kernel<kMidCap, 512><<<256, 512, 0, st>>>(
      a.counts, a.caps, a.rstart, a.soff, a.smap, a.slots, lay.cap_slots, offsets, a.RW, key_bytes, a.out,
      reinterpret_cast<const uint32_t*>(part + lay.mid_list), &a.ph->n_mid, B);
  bucket_sort_global_kernel<<<256, kBigThreads, 0, st>>>(a.counts, a.caps, a.rstart, a.soff, a.smap, a.slots,
                                                         lay.cap_slots, offsets, a.RW, key_bytes, a.out,
                                                         reinterpret_cast<const uint32_t*>(part + lay.big_list),
                                                         &a.ph->n_big);
  return hipGetLastError();
}

}  // namespace elsar
