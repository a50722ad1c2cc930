// Seeded synthetic record generator on the GPU (input generator only).
//
// The same records as gen.c, byte for byte, written straight into device
// memory: every byte is the same pure function of (seed, record index) through
// Philox4x32-10 (Salmon et al., SC'11) with the same counter layout
// {idx_lo, idx_hi, stream, block} and key {seed_lo, seed_hi}.  It exists so
// that data sets of hundreds of GB can be laid out in HBM, and restored
// between in-place runs, without a trip through host memory.  It holds none
// of the sorting method's arithmetic.  The rank-law thresholds (inverse CDF
// tables) come from the host library, so the floating-point law construction
// happens in one place only.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

struct Spec {  // same fields and meaning as gen_spec in gen.c
  uint32_t kind, record_bytes, key_bytes, embed_idx;
  uint64_t seed;
  double mean_rank, sigma, hot_fraction;
  uint32_t n_hot, stair_bytes;
  double zipf_s, mix_p;
};

struct Laws {
  uint64_t normal[95];
  uint64_t zipf[95];
};

// Law tables of the current call (copied synchronously before each launch;
// calls in flight on other streams must use the same laws).
__constant__ Laws c_laws;

enum { UNIFORM = 0, NORMAL_HOT = 1, ZIPF_FIRST = 2, MIX = 3, STAIRCASE = 4 };
enum { S_KEY = 0, S_PAYLOAD = 1, S_CHOICE = 2, S_HOT = 3, S_STAIR = 5 };

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 draw(uint64_t seed, uint64_t idx, uint32_t stream, uint32_t block) {
  uint32_t c0 = (uint32_t)idx, c1 = (uint32_t)(idx >> 32), c2 = stream, c3 = block;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c1 = lo1; c3 = lo0; c0 = n0; c2 = n2;
  }
  return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t pick(const U4& u, uint32_t i) {
  return i == 0 ? u.x : (i == 1 ? u.y : (i == 2 ? u.z : u.w));
}

__device__ __forceinline__ uint32_t rank_from(const uint64_t* thr, uint32_t u) {
  int lo = 0, hi = 94;  // smallest r with u < thr[r]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((uint64_t)u < thr[mid]) hi = mid; else lo = mid + 1;
  }
  return (uint32_t)lo;
}

__device__ __forceinline__ uint32_t uniform_char(uint32_t u) {
  return 0x20u + (uint32_t)(((uint64_t)u * 95u) >> 32);
}

// One thread per record; the record is assembled four bytes at a time.
__global__ void gen_kernel(Spec sp, uint64_t start, uint64_t count, uint32_t* __restrict__ out) {
  const uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (t >= count) return;
  const uint64_t idx = start + t;
  const uint32_t R = sp.record_bytes, K = sp.key_bytes;
  const U4 ch = draw(sp.seed, idx, S_CHOICE, 0);
  uint32_t kind = sp.kind;
  if (kind == MIX) kind = ((double)ch.z < sp.mix_p * 4294967296.0) ? UNIFORM : NORMAL_HOT;
  // where the key bytes come from
  uint64_t kidx = idx;
  uint32_t kstream = S_KEY;
  const uint64_t* law0 = nullptr;
  const uint64_t* law_rest = nullptr;
  if (kind == ZIPF_FIRST) {
    law0 = c_laws.zipf;
  } else if (kind == NORMAL_HOT) {
    law0 = law_rest = c_laws.normal;
    if ((double)ch.x < sp.hot_fraction * 4294967296.0) {
      const uint32_t n_hot = sp.n_hot ? sp.n_hot : 1u;
      kidx = ((uint64_t)ch.y * n_hot) >> 32;
      kstream = S_HOT;
    }
  }
  const uint32_t sb = sp.stair_bytes < K ? sp.stair_bytes : K;
  const bool stair = kind == STAIRCASE && idx > 0;
  const uint64_t row = stair ? (uint64_t)((63u - (uint32_t)__clzll((long long)idx)) % 128u) : 0ull;
  uint32_t* o = out + t * (R / 4);
  U4 ku{}, su{}, pu{};
  uint32_t word = 0;
  for (uint32_t b = 0; b < R; ++b) {
    uint32_t c;
    if (b < K) {
      if ((b & 3u) == 0) {
        ku = draw(sp.seed, kidx, kstream, b >> 2);
        if (stair) su = draw(sp.seed, row, S_STAIR, b >> 2);
      }
      if (stair && b < sb) {
        c = uniform_char(pick(su, b & 3u));
      } else {
        const uint32_t v = pick(ku, b & 3u);
        const uint64_t* law = b == 0 ? law0 : law_rest;
        c = law ? 0x20u + rank_from(law, v) : uniform_char(v);
      }
    } else {
      const uint32_t pb = b - K;
      if ((pb & 15u) == 0) pu = draw(sp.seed, idx, S_PAYLOAD, pb >> 4);
      if (sp.embed_idx && pb < 10) {  // the index as 10 decimal digits over the payload's start
        uint64_t v = idx;
        for (uint32_t d = 9; d > pb; --d) v /= 10;
        c = (uint32_t)('0' + v % 10);
      } else {
        const uint32_t byte = (pick(pu, (pb >> 2) & 3u) >> (8 * (pb & 3u))) & 0xFFu;
        c = 0x20u + ((byte * 95u) >> 8);
      }
    }
    word |= c << (8 * (b & 3u));
    if ((b & 3u) == 3u) {
      o[b >> 2] = word;
      word = 0;
    }
  }
}

}  // namespace

// Records start .. start+count-1 into device memory d_out (4-byte aligned,
// record_bytes a multiple of 4); thresholds as gen_rank_law returns them.
extern "C" int gen_records_device(const Spec* sp, const uint64_t* thr_normal, const uint64_t* thr_zipf,
                                  uint64_t start, uint64_t count, void* d_out, hipStream_t stream) {
  if (!sp || !d_out || sp->record_bytes == 0 || sp->record_bytes % 4 != 0 || sp->key_bytes == 0 ||
      sp->key_bytes > sp->record_bytes || sp->kind > STAIRCASE)
    return 1;
  if (sp->embed_idx && sp->record_bytes < sp->key_bytes + 10) return 1;
  if ((reinterpret_cast<uintptr_t>(d_out) & 3u) != 0) return 1;
  if (count == 0) return 0;
  Laws laws;
  for (int r = 0; r < 95; ++r) {
    laws.normal[r] = thr_normal[r];
    laws.zipf[r] = thr_zipf[r];
  }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_laws), &laws, sizeof(laws), 0, hipMemcpyHostToDevice) != hipSuccess) return 2;
  const uint64_t blocks = (count + 255) / 256;
  gen_kernel<<<(uint32_t)blocks, 256, 0, stream>>>(*sp, start, count, static_cast<uint32_t*>(d_out));
  return hipGetLastError() == hipSuccess ? 0 : 2;
}
