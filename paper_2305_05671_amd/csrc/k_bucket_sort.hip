// In-bucket sort and concatenation (gfx950): Section 3.4 (sort each partition)
// and Section 3.5 (write it at the exclusive prefix sum of the partition sizes,
// coalescing the records in sorted order).
//
// A bucket's records sit in its region (and possibly the spill area).  Each is
// reduced to a 16-byte sort entry: the key bytes and then the 32-bit input
// index, as one big-endian composite, so sorting the composites orders by
// key in memcmp order and breaks ties by input position.  An LSD radix sort
// with 8-bit digits runs over the composite's bytes, skipping every byte that
// is equal across the whole bucket (an all-equal-key bucket only sorts its
// index bytes).  The records are then copied in sorted order to
// out + R * offsets[j] with dword stores contiguous across lanes.
//
//  * bucket_sort_lds<CAP, THREADS>: one block per bucket of at most CAP records;
//    entries and the permutation live in LDS.
//  * bucket_sort_global: buckets above the larger cap, one block each; the
//    ping-pong entry buffers live in the bucket's own output range, which holds
//    R*n bytes and is not yet written (R >= 40 gives 2 * 20n bytes of room).
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

// Composite sort key of a slot: key bytes [0, K) then the index, big-endian,
// as four words (word 0 most significant).  Bytes beyond K+4 are zero.
__device__ __forceinline__ uint4 composite(const uint32_t* __restrict__ s, uint32_t W, uint32_t K) {
  uint32_t w0 = s[0], w1 = s[1], w2 = s[2], idx = s[W - 1];
  uint32_t tb = K - 8;  // key bytes in the third word, 0..4
  uint32_t t = __builtin_bswap32(w2);
  t = tb == 0 ? 0u : (tb >= 4 ? t : (t & (0xFFFFFFFFu << (32 - 8 * tb))));
  uint64_t low = ((uint64_t)t << 32) | ((uint64_t)idx << (32 - 8 * tb));
  return make_uint4(__builtin_bswap32(w0), __builtin_bswap32(w1), (uint32_t)(low >> 32), (uint32_t)low);
}

__device__ __forceinline__ uint32_t digit_of(const uint4& c, uint32_t p) {
  uint32_t w = p < 4 ? c.x : (p < 8 ? c.y : (p < 12 ? c.z : c.w));
  return (w >> (24 - 8 * (p & 3))) & 0xFFu;
}

// OR and AND across the block; *vary gets the composite bytes that differ.
template <uint32_t THREADS>
__device__ uint32_t varying_bytes(uint4 o, uint4 a, uint4* sh_or, uint4* sh_and) {
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
  uint4 d = make_uint4(O.x ^ A.x, O.y ^ A.y, O.z ^ A.z, O.w ^ A.w);
  uint32_t vary = 0;
  for (uint32_t p = 0; p < 16; ++p) vary |= (uint32_t)(digit_of(d, p) != 0) << p;
  __syncthreads();
  return vary;
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
    // inclusive scan of run over the 4 waves of the first 256 threads
    uint32_t v = run;
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

template <uint32_t CAP, uint32_t THREADS>
__global__ __launch_bounds__(THREADS) void bucket_sort_lds_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps, const uint32_t* __restrict__ rstart,
    const uint32_t* __restrict__ spill_off, const uint32_t* __restrict__ spill_map,
    const uint32_t* __restrict__ slots, uint64_t cap_slots, const uint64_t* __restrict__ offsets, uint32_t RW,
    uint32_t K, uint32_t* __restrict__ out, const uint32_t* __restrict__ list, const uint32_t* __restrict__ list_n,
    uint32_t B) {
  constexpr uint32_t WAVES = THREADS / 64;
  constexpr uint32_t ROUNDS = CAP / THREADS;
  static_assert(CAP % THREADS == 0, "cap is whole rounds");
  __shared__ uint4 ent[CAP];
  __shared__ uint16_t perm[2][CAP];
  __shared__ uint32_t wc[WAVES][256];
  __shared__ uint4 sh_or[WAVES], sh_and[WAVES];
  __shared__ uint32_t tot[4];
  const uint32_t W = RW + 1;
  const uint32_t w = threadIdx.x >> 6;
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
      uint4 c = composite(slots + (uint64_t)sl * W, W, K);
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
      for (uint32_t i = threadIdx.x; i < WAVES * 256; i += THREADS) (&wc[0][0])[i] = 0;
      __syncthreads();
      uint32_t dg[ROUNDS], lc[ROUNDS];
      uint16_t ev[ROUNDS];
#pragma unroll
      for (uint32_t r = 0; r < ROUNDS; ++r) {
        uint32_t i = w * (ROUNDS * 64) + r * 64 + lane_id();
        bool valid = i < br.n;
        uint16_t e = valid ? perm[cur][i] : 0;
        uint32_t d = valid ? digit_of(ent[e], (uint32_t)pbyte) : 0u;
        uint64_t peers = match_digit8(d, valid);
        uint32_t rank = __popcll(peers & lanemask_lt());
        uint32_t prev = valid ? wc[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wc[w][d] = prev + (uint32_t)__popcll(peers);
        __builtin_amdgcn_wave_barrier();
        dg[r] = d;
        lc[r] = prev + rank;
        ev[r] = e;
      }
      __syncthreads();
      digit_wave_offsets<WAVES>(wc, tot);
      __syncthreads();
#pragma unroll
      for (uint32_t r = 0; r < ROUNDS; ++r) {
        uint32_t i = w * (ROUNDS * 64) + r * 64 + lane_id();
        if (i < br.n) perm[cur ^ 1][wc[w][dg[r]] + lc[r]] = ev[r];
      }
      __syncthreads();
      cur ^= 1;
    }
    // 3. copy records in sorted order to the output
    const uint32_t total = br.n * RW;
    uint32_t* o_dw = out + br.out0 * RW;
    for (uint32_t f = threadIdx.x; f < total; f += THREADS) {
      uint32_t k = f / RW, d = f - k * RW;
      uint32_t sl = slot_of(br, perm[cur][k], spill_map, cap_slots);
      o_dw[f] = slots[(uint64_t)sl * W + d];
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
  const uint32_t W = RW + 1;
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
    uint32_t* o_dw = out + br.out0 * RW;           // R*n bytes = RW*n dwords
    uint32_t* buf0 = o_dw + (uint64_t)(RW - 10) * br.n;  // (R-40)*n bytes in
    uint32_t* buf1 = o_dw + (uint64_t)(RW - 5) * br.n;   // (R-20)*n bytes in
    // 1. which composite bytes vary
    uint4 o = make_uint4(0, 0, 0, 0), a = make_uint4(~0u, ~0u, ~0u, ~0u);
    for (uint32_t p = threadIdx.x; p < br.n; p += kBigThreads) {
      uint4 c = composite(slots + (uint64_t)slot_of(br, p, spill_map, cap_slots) * W, W, K);
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
      put_entry(cur, p, composite(slots + (uint64_t)sl * W, W, K), sl);
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
        o_dw[(uint64_t)k0 * RW + f] = slots[(uint64_t)chunk_slot[k] * W + d];
      }
      __syncthreads();
    }
  }
}

hipError_t launch_bucket_sort(const uint8_t* part, const PartLayout& lay, uint32_t B, const uint64_t* offsets,
                              uint32_t rec_bytes, uint32_t key_bytes, uint8_t* out, hipStream_t st) {
  const uint32_t RW = rec_bytes / 4;
  auto* counts = reinterpret_cast<const uint32_t*>(part + lay.counts);
  auto* caps = reinterpret_cast<const uint32_t*>(part + lay.caps);
  auto* rstart = reinterpret_cast<const uint32_t*>(part + lay.rstart);
  auto* soff = reinterpret_cast<const uint32_t*>(part + lay.spill_off);
  auto* smap = reinterpret_cast<const uint32_t*>(part + lay.spill_map);
  auto* slots = reinterpret_cast<const uint32_t*>(part + lay.slots);
  auto* ph = reinterpret_cast<const PartHeader*>(part + lay.header);
  auto* o = reinterpret_cast<uint32_t*>(out);
  bucket_sort_lds_kernel<kSmallCap, 256><<<B, 256, 0, st>>>(counts, caps, rstart, soff, smap, slots, lay.cap_slots,
                                                             offsets, RW, key_bytes, o, nullptr, nullptr, B);
  bucket_sort_lds_kernel<kMidCap, 512><<<256, 512, 0, st>>>(
      counts, caps, rstart, soff, smap, slots, lay.cap_slots, offsets, RW, key_bytes, o,
      reinterpret_cast<const uint32_t*>(part + lay.mid_list), &ph->n_mid, B);
  bucket_sort_global_kernel<<<256, kBigThreads, 0, st>>>(counts, caps, rstart, soff, smap, slots, lay.cap_slots,
                                                         offsets, RW, key_bytes, o,
                                                         reinterpret_cast<const uint32_t*>(part + lay.big_list),
                                                         &ph->n_big);
  return hipGetLastError();
}

}  // namespace elsar
