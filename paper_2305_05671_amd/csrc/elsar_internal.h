// Internal declarations of the HIP/gfx950 ELSAR library: device data layouts,
// device helpers shared by the kernels, and host launch wrappers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace elsar {

// ---------------------------------------------------------------- layout --
// One partition slot: the record's 32-bit input index, then the record, zero
// padding up to a whole number of 128-byte lines (one line for 100-byte
// records).  A slot is written as full lines, so no write leaves a partial
// line for the memory side to merge.  Its first 16 bytes hold the index and
// the first 12 record bytes, so one load gives the whole sort key.  The index
// makes the in-bucket order independent of the order in which the atomics
// handed out slots.
constexpr uint32_t kMaxKeyBytes = 28;   // bytes 12.. of a longer key order runs of equal 12-byte prefixes
constexpr uint32_t kSortKeyBytes = 12;  // the bucket sorts' entry holds key bytes 0..11 + the 4-byte index
constexpr uint32_t kMinKeyBytes = 8;    // the code reads the first 8 key bytes
constexpr uint32_t kSmallCap = 2048;    // largest bucket sorted by the small LDS kernel
constexpr uint32_t kMidCap = 6144;      // largest bucket sorted by the large LDS kernel
constexpr uint32_t kMidLoCap = 3072;    // its half-size instance (two blocks per CU) takes buckets up to here
constexpr uint32_t kMaxBuckets = 1u << 21;

struct Leaf {          // one RMI leaf: clamped line on the leaf-local code
  uint64_t base;       // smallest sample code routed to the leaf
  float c, b;          // slope (>= 0), intercept, bucket units
  uint32_t lo, hi;     // bucket range the leaf's own sample ranks span
  uint32_t pad[2];
};
static_assert(sizeof(Leaf) == 32, "leaf is two 16-byte vectors");

struct ModelHeader {   // device-resident root of a fitted model
  float a0, a1;        // linear root in leaf units
  uint32_t L, B;       // leaves, buckets
  uint32_t kind_used;  // root in use: 0 = linear RMI, 1 = MLP, 2 = linear spline
  uint32_t mlp_rejected;
  uint64_t n_fit;      // records the model was fitted for
  uint64_t S;          // sample size
  uint32_t max_sample_bucket, opt_sample_bucket;
  uint32_t max_sample_run;  // longest run of equal codes in the sorted sample
  uint32_t mlp_L;           // equi-depth leaves under the MLP or spline root
  uint32_t mlp_skip;        // automatic choice: the linear root passed the gate
  uint32_t spline_K;        // segments of the spline root
  // acceptance statistics: largest sample bucket under the linear root, under
  // the equi-depth leaves, and under the network's own buckets
  // clamp(floor(B y), 0, B-1); whether the linear root passed its gate; the
  // gate's bound lambda + sqrt(2 ln(B) lambda) + 1, lambda = S/B
  uint32_t max_rmi, max_eq, max_net, rmi_ok;
  float perfect;
  uint32_t cell_shift;  // equi-depth leaves: code-cell width 2^cell_shift (code_cell)
  uint32_t pad_[2];
};

// Monotone MLP root (8 -> 64 -> 64 -> 1), flat parameter order W1 (64x8),
// b1, W2 (64x64), b2, w3, b3.
constexpr uint32_t kMlpH = 64;
constexpr uint32_t kOffW1 = 0, kOffB1 = 512, kOffW2 = 576, kOffB2 = 4672, kOffW3 = 4736, kOffB3 = 4800;
constexpr uint32_t kMlpParams = 4801;

struct MlpHead {       // what the vector ALUs read: knots and the FP32 layers
  uint64_t q[9];       // knots: codes at the sample's 1/8 quantiles, and the largest
  float inv_w[8];      // 1 / max(q[k+1] - q[k], 1)
  float W1[512];       // [unit][feature]
  float b1[64], b2[64], w3[64];
  float b3;
  float pad[3];
};
// Rows of the bfloat16 W2 copies are kW2S entries apart (64 and a pad of 4):
// the 16 lanes of a matrix-core fragment read 16 consecutive rows, which then
// fall in different LDS banks where a block keeps the copies in LDS.
constexpr uint32_t kW2S = 68;
struct MlpBlock {      // evaluation copy of the parameters
  MlpHead h;
  uint16_t W2bf[64 * kW2S];   // bfloat16 W2[j][u] at [j * kW2S + u]
  uint16_t W2bfT[64 * kW2S];  // bfloat16 W2[j][u] at [u * kW2S + j]
};
static_assert(sizeof(MlpHead) % 8 == 0, "W2 copies stay 8-byte aligned");

struct PartHeader {    // device-resident state of one partition pass
  uint64_t n;
  uint64_t cap_slots;   // slots reserved for bucket regions (upper bound)
  uint32_t B;
  uint32_t spill_count; // records that overflowed their region
  uint32_t n_mid;       // buckets with kSmallCap < count <= kMidLoCap (listed from the start of mid_list)
  uint32_t n_big;       // buckets with count > kMidCap
  uint32_t max_count;
  uint32_t mid_records;  // records in the n_mid buckets
  uint32_t big_records;  // records in the n_big buckets
  uint32_t seg_n[4];     // split of the n_big buckets: segments, stack overflow flag, spare (2)
  uint32_t n_big2;       // of the n_big buckets, those the equal-key kernel leaves to the split
  uint32_t n_mid_hi;     // of the n_mid buckets, those above kMidLoCap (listed from the end of mid_list)
  uint32_t pad;
};

// From kScanMultiMin buckets up, the region sizes and the count scan of one
// job run over chunks of kScanChunk buckets, one block each, in two launches;
// a chunk's sums pass between them as a ScanPart.
constexpr uint32_t kScanChunk = 4096;
constexpr uint32_t kScanMultiMin = 16384;
struct ScanPart {
  uint64_t c;  // sizes or counts of the chunk's buckets
  uint32_t s;  // their records beyond the regions
  uint32_t pad;
};

// Byte offsets of the partition buffer's parts for n records and B buckets.
struct PartLayout {
  size_t header, counts, caps, rstart, spill_off, mid_list, big_list;
  size_t psum;       // one ScanPart per chunk of kScanChunk buckets
  size_t big2_list;  // the big buckets left to the split (keys not all equal, or above the equal-key cap)
  // The partition's slot counters: bucket j's at pcounts + 4 * j * cstride.
  // Returning atomics on counters packed 32 to a 128-byte line serialise per
  // line (10^6 of them on 1024 packed counters took 5x as long as on the same
  // counters one per line), so with fewer than 65536 buckets the counters are
  // spread over at least 2048 lines; the scan then writes the dense counts
  // the bucket sorts read.  With cstride 1, pcounts == counts.
  size_t pcounts;
  uint32_t cstride;
  size_t spill_meta, spill_map, slots;
  size_t seg_leaf;               // segment list of the big-bucket split
  uint32_t seg_leaf_cap;
  uint64_t cap_slots;   // region slots
  uint64_t total_slots; // regions + spill
  size_t bytes;
  uint32_t slot_bytes;  // slot_bytes_for(record_bytes)
};

__host__ __device__ constexpr uint32_t slot_bytes_for(uint32_t rec_bytes) { return (rec_bytes + 4 + 127) / 128 * 128; }

// Spacing (in u32) of the partition's slot counters for B buckets.  Every
// record is one atomic on its bucket's counter, and atomics to one 128-byte
// line serialise in L2, so with few buckets the counters are spread over at
// least 2048 lines (at most one per line).  From 65536 buckets up they stay
// dense: the counters are already spread over enough lines, and padding
// them only adds L2 footprint.
inline uint32_t counter_stride(uint32_t B) {
  if (B >= 65536) return 1;
  const uint32_t s = 65536 / B;
  return s < 32 ? s : 32;
}

// ----------------------------------------------------------- device code --
// Native 4 x u32 vector for register-held data: HIP's uint4 struct copies go
// through memcpy, which can pin the value in scratch memory.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t philox_x(uint64_t ctr_lo64, uint32_t c2, uint32_t c3, uint64_t key) {
  // Philox4x32-10 (Salmon et al., SC'11); only the first output word is used.
  uint32_t c0 = (uint32_t)ctr_lo64, c1 = (uint32_t)(ctr_lo64 >> 32);
  uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c1 = lo1; c3 = lo0; c0 = n0; c2 = n2;
  }
  return c0;
}

// Base-95 code of the first 8 key bytes (little-endian dwords w0 = bytes 0..3,
// w1 = bytes 4..7).  From the first byte outside 0x20..0x7E on, every digit
// saturates to 0 (byte below 0x20) or 94 (above 0x7E): non-decreasing in
// memcmp order for any bytes.  Two 4-digit halves, each < 95^4 < 2^27.
__device__ __forceinline__ uint64_t key_code(uint32_t w0, uint32_t w1) {
  uint32_t bad = 0, low = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint32_t c = ((i < 4 ? w0 : w1) >> (8 * (i & 3))) & 0xFFu;
    bad |= (uint32_t)(c < 0x20u || c > 0x7Eu) << i;
    low |= (uint32_t)(c < 0x20u) << i;
  }
  uint32_t p = bad ? (uint32_t)__builtin_ctz(bad) : 8u;
  uint32_t sat = ((low >> p) & 1u) ? 0u : 94u;
  uint32_t h = 0, l = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint32_t c = ((i < 4 ? w0 : w1) >> (8 * (i & 3))) & 0xFFu;
    uint32_t d = (uint32_t)i < p ? c - 0x20u : sat;
    if (i < 4) h = h * 95u + d; else l = l * 95u + d;
  }
  return (uint64_t)h * 81450625ull + l;  // 95^4
}

// Variable-length keys.  vk = 0: fixed-length keys.  Otherwise vk = (lo << 8)
// | K: the key field is record bytes [0, K) (K <= 11), the key proper is its
// first len bytes, len = min(record byte lo, K) with K <= lo < 12, and the
// field's bytes from len on are padding, whatever they hold.  Order: the
// padded key with the padding read as 0x00 (below every byte value), then
// len, so that a key sorts before the keys it is a proper prefix of.  The
// record's first 12 bytes (little-endian dwords r0..r2) become that sort key
// as a fixed key of K + 1 bytes: bytes [0, len) kept, [len, K) zero, byte K =
// len, the rest zero.  Every kernel that reads a key applies this first, so
// the code, the bucket and the composite all see the same key.
__device__ __forceinline__ void virtual_key(uint32_t& r0, uint32_t& r1, uint32_t& r2, uint32_t vk) {
  if (!vk) return;
  const uint32_t K = vk & 0xFFu, lo = vk >> 8;
  const uint32_t w = lo < 4 ? r0 : (lo < 8 ? r1 : r2);
  uint32_t len = (w >> (8 * (lo & 3u))) & 0xFFu;
  len = len < K ? len : K;
  auto keep = [&](uint32_t x, uint32_t base) -> uint32_t {  // bytes base..base+3 of the window
    if (len >= base + 4) return x;
    if (len <= base) return 0u;
    return x & ((1u << (8 * (len - base))) - 1u);
  };
  r0 = keep(r0, 0);
  r1 = keep(r1, 4);
  r2 = keep(r2, 8) | (len << (8 * (K - 8)));  // K in 8..11: byte K sits in r2
}

__device__ __forceinline__ float code_f32(uint64_t e) { return (float)(double)e; }

__device__ __forceinline__ uint32_t rmi_leaf(float a0, float a1, uint32_t L, uint64_t e) {
  float r = floorf(__builtin_fmaf(a1, code_f32(e), a0));
  if (r < 0.0f) return 0;
  if (r > (float)(L - 1)) return L - 1;
  return (uint32_t)r;
}

// The clamp to [lo, hi] is written without branches (lo and hi are bucket ids,
// exact in FP32, and y is finite): with an early return the compiler deferred
// the load of hi behind the test on lo, a second dependent trip to L2 for
// nearly every record.
__device__ __forceinline__ uint32_t leaf_bucket(const Leaf& lf, uint64_t e) {
  uint64_t d = e >= lf.base ? e - lf.base : 0;
  const float y = floorf(__builtin_fmaf(lf.c, code_f32(d), lf.b));
  return (uint32_t)fminf(fmaxf(y, (float)lf.lo), (float)lf.hi);
}

// Spline root over equi-depth leaves: K segments of about L / K leaves each;
// segment i holds leaves (i L) / K .. ((i + 1) L) / K - 1 and starts at the
// code knots[i] = bound[(i L) / K] (knots[K] past every code).
__host__ __device__ __forceinline__ uint32_t spline_segments(uint32_t L) { return L >= 64 ? L / 64 : 1; }

// Routing to an equi-depth leaf: the last leaf j with bound[j] <= code (leaf
// 0 below bound[1]).  A table over the code range narrows the search: with NC
// cells (code_cells_for(L)), cell c holds the codes e with
// (e - bound[1]) >> cell_shift == c (codes at or below bound[1] in cell 0,
// codes past the last cell in the last), cell_shift the smallest with
// (bound[L-1] - bound[1]) >> cell_shift < NC, and ccells[c] counts the
// boundaries bound[1 .. L-1] in cells below c.  Cells are monotone in the
// code, so a code of cell c lies in a leaf j with ccells[c] <= j <=
// ccells[c + 1]: the search covers the boundaries that share the code's cell.
// There is about one cell per leaf (at least 1024, at most 2^18 cells):
// where the codes are spread evenly a cell holds a boundary or two and one
// or two probes name the leaf (against about 16 for a search over segment
// knots then leaves).  Where the keys are dense in code space (the skewed
// law's per-byte peaks put tens of boundaries in one cell), a cell with
// more than kCellDense boundaries has a sub-table of
// 2^k cells of its own (2^k at least twice its boundaries, k at most
// cell_shift): entry s counts the boundaries below its sub-cell s, exactly as
// the cells do, so the search narrows to the boundaries of the code's
// sub-cell.  Layout (32-bit words): per cell c a pair {ccells[c], info[c]},
// info = (((sub-table offset << 5) | k) << 1) | 1 with a sub-table, else the
// cell's own boundary count ccells[c + 1] - ccells[c] shifted left by one (so
// a record in a cell without a sub-table reads one pair, not the next cell's
// too: the compiler had deferred that load behind the test on info), for c =
// 0..NC (the pair NC holds the boundary count only), then the sub-tables: cell c's at
// offset 4 ccells[c] + c, 2^k + 1 <= 4 (ccells[c + 1] - ccells[c]) entries
// (2^k < 4 x the cell's boundaries), so the tables never overlap and fit in
// 4 L + NC + 1 words without any allocation step.
constexpr uint32_t kCellDense = 3;

__host__ __device__ __forceinline__ uint32_t code_cells_for(uint32_t L) {
  uint32_t nc = 1024;
  while (nc < L && nc < (1u << 18)) nc <<= 1;
  return nc;
}

__host__ __device__ __forceinline__ size_t cell_table_words(uint32_t L) {
  const size_t nc = code_cells_for(L);
  return 2 * (nc + 1) + 4 * (size_t)L + nc + 1;
}

__host__ __device__ __forceinline__ uint32_t code_cell(uint64_t e, uint64_t e0, uint32_t shift, uint32_t nc) {
  const uint64_t d = e > e0 ? (e - e0) >> shift : 0ull;
  return d < nc ? (uint32_t)d : nc - 1;
}

// Sub-cell of a code in dense cell c (codes below bound[1] in sub-cell 0,
// codes past the cell in its last).
__host__ __device__ __forceinline__ uint32_t code_subcell(uint64_t e, uint64_t e0, uint32_t shift, uint32_t c,
                                                          uint32_t k) {
  const uint64_t d = e > e0 ? (e - e0) >> (shift - k) : 0ull;
  const uint64_t rel = d - ((uint64_t)c << k);  // d >= c << k: the code's cell is c or it was clamped to c
  return rel < (1ull << k) ? (uint32_t)rel : (1u << k) - 1u;
}

__device__ __forceinline__ uint32_t cell_exact_leaf(const uint32_t* __restrict__ ccells, uint32_t shift,
                                                    uint32_t nc, uint64_t e0, const uint64_t* __restrict__ bound,
                                                    uint64_t code) {
  const uint32_t c = code_cell(code, e0, shift, nc);
  const uint2* cl = reinterpret_cast<const uint2*>(ccells);
  const uint2 x = cl[c];
  uint32_t a = x.x, b = x.x + (x.y >> 1);
  if (x.y & 1u) {
    const uint32_t k = (x.y >> 1) & 31u;
    const uint32_t* sub = ccells + 2 * ((size_t)nc + 1) + (x.y >> 6);
    const uint32_t s = code_subcell(code, e0, shift, c, k);
    a = sub[s];
    b = sub[s + 1];
  }
  b += 1;  // bound[a] <= code < bound[b] (bound[L] never read)
  while (b - a > 1) {
    const uint32_t mid = (a + b) >> 1;
    if (bound[mid] <= code) a = mid; else b = mid;
  }
  return a;
}

__device__ __forceinline__ Leaf load_leaf(const Leaf* __restrict__ leaves, uint32_t j) {
  const uint4* p = reinterpret_cast<const uint4*>(leaves + j);
  uint4 a = p[0], b = p[1];
  Leaf lf;
  lf.base = (uint64_t)a.x | ((uint64_t)a.y << 32);
  lf.c = __uint_as_float(a.z);
  lf.b = __uint_as_float(a.w);
  lf.lo = b.x;
  lf.hi = b.y;
  return lf;
}

// Lanes of the wave holding the same 8-bit digit as this lane (valid lanes only).
__device__ __forceinline__ uint64_t match_digit8(uint32_t d, bool valid) {
  uint64_t m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    bool bit = (d >> b) & 1u;
    uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int off) {
  uint32_t lo = __shfl_xor((uint32_t)v, off), hi = __shfl_xor((uint32_t)(v >> 32), off);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int off) {
  uint32_t lo = __shfl_up((uint32_t)v, off), hi = __shfl_up((uint32_t)(v >> 32), off);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = __shfl((uint32_t)v, src), hi = __shfl((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// Inclusive scan of one value per lane across a whole (converged) wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  T x = v;
  for (int off = 1; off < 64; off <<= 1) {
    T y;
    if constexpr (sizeof(T) == 8) y = (T)shfl_up_u64((uint64_t)x, off);
    else y = (T)__shfl_up((uint32_t)x, off);
    if (lane_id() >= (uint32_t)off) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread across a block of NT threads (NT a
// multiple of 64, at most 1024).  *total gets the block's sum.  sh: NT/64 slots.
template <typename T, uint32_t NT>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sh, T* total) {
  T x = v;
  for (int off = 1; off < 64; off <<= 1) {
    T y;
    if constexpr (sizeof(T) == 8) y = (T)shfl_up_u64((uint64_t)x, off);
    else y = (T)__shfl_up((uint32_t)x, off);
    if (lane_id() >= (uint32_t)off) x += y;
  }
  const uint32_t w = threadIdx.x >> 6;
  if (lane_id() == 63) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (uint32_t i = 0; i < NT / 64; ++i) {
      T c = sh[i];
      sh[i] = run;
      run += c;
    }
    sh[NT / 64] = run;
  }
  __syncthreads();
  T r = sh[w] + x - v;
  *total = sh[NT / 64];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------- host wrappers --
// sample / fit (k_fit.hip)
hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st);
hipError_t launch_sample_codes(const uint8_t* recs, uint64_t n, uint32_t rec_bytes, uint64_t S, uint64_t seed,
                               uint64_t* codes, hipStream_t st, uint32_t vk = 0);
size_t radix_u64_scratch_bytes(uint64_t n);
hipError_t launch_radix_sort_u64(uint64_t* keys, uint64_t* tmp, uint64_t n, int lo_byte, int hi_byte,
                                 void* scratch, hipStream_t st, uint64_t** sorted);
size_t fit_scratch_bytes(uint64_t S);
hipError_t launch_fit_rmi(const uint64_t* sorted_codes, uint64_t S, uint64_t n, uint32_t L, uint32_t B,
                          ModelHeader* hdr, Leaf* leaves, void* scratch, hipStream_t st);
hipError_t launch_sample_hist(const ModelHeader* hdr, const Leaf* leaves, const uint64_t* sorted_codes,
                              uint64_t S, uint32_t B, uint32_t* hist, hipStream_t st);
// batch: one block fits the linear model of one job; a sample of up to
// kBatchFitMaxS codes is sorted in LDS, one of up to kBatchFitChunks times
// that in chunks through 2 S codes of global scratch
constexpr uint64_t kBatchFitMaxS = 16384;
constexpr uint64_t kBatchFitChunks = 3;
struct FitJob {
  const uint8_t* recs;   // the job's records (device)
  uint64_t n, S, seed;
  uint32_t L, B;
  ModelHeader* hdr;
  Leaf* leaves;          // L
  uint32_t* hist;        // B
  uint64_t* scratch;     // 2 S codes when S > kBatchFitMaxS, else unused
};
hipError_t launch_batch_fit(const FitJob* d_jobs, uint32_t njobs, uint32_t rec_bytes, hipStream_t st);
hipError_t launch_radix_model(uint64_t S, uint64_t n, uint32_t L, uint32_t B, ModelHeader* hdr, Leaf* leaves,
                              hipStream_t st);
hipError_t launch_capacities(const uint32_t* hist, uint64_t S, uint64_t n, uint32_t B, uint32_t region_pct,
                             uint8_t* part, const PartLayout& lay, hipStream_t st);

// Equi-depth roots (k_mlp.hip): the MLP and the linear spline share leaves
// cut at sample quantiles; the state beyond the RMI's.
struct MlpState {
  MlpBlock* M;
  Leaf* leaves;      // L equi-depth leaves
  uint64_t* bound;   // L + 1 routing boundaries: leaf j takes codes in [bound[j], bound[j+1])
  uint32_t* first;   // L + 1: first sample rank of each leaf
  uint32_t* hist;    // B: sample keys per bucket under these leaves
  uint32_t* hist_net;  // B: sample keys per bucket of the network's own output, floor(B y)
  uint64_t* knots;   // spline_segments(L) + 1 segment knots of the spline root
  uint32_t* ccells;  // code_cells_for(L) + 1: the code-cell table that brackets the leaf search
  uint32_t* cells;   // L + 1: cells[c] = leaves whose MLP cell floor(L y(bound[j])) is below c
  float* master;     // kMlpParams FP32 parameters of the MLP
  float* adam;       // 2 * kMlpParams moments
};
size_t mlp_state_bytes(uint32_t L, uint32_t B);
void place_mlp_state(MlpState* s, void* base, uint32_t L, uint32_t B);
// MLP training on the sorted sample (initial weights, Adam steps).
hipError_t launch_mlp_train(const uint64_t* sorted_codes, uint64_t S, uint64_t seed, uint32_t steps, float lr,
                            const MlpState& ms, hipStream_t st);
// Histogram of the trained network's own buckets clamp(floor(B y), 0, B-1)
// over the sorted sample (the MLP's acceptance statistic).
hipError_t launch_mlp_net_hist(const MlpState& ms, const uint64_t* sorted_codes, uint64_t S, uint32_t B,
                               hipStream_t st);
// Key bytes the bucket sorts order by; a longer key is finished by the run fix-up.
inline uint32_t sort_key_bytes(uint32_t K) { return K < kSortKeyBytes ? K : kSortKeyBytes; }
// Keys longer than kSortKeyBytes: device scratch of the run fix-up for n
// records, and the fix-up itself on n sorted records at `out` (in place).
size_t long_key_scratch_bytes(uint64_t n, uint32_t rec_bytes);
hipError_t launch_long_key_fixup(uint8_t* out, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes, uint8_t* scratch,
                                 hipStream_t st);
// Equi-depth leaves, their splines and boundaries, the spline root's knots,
// and the sample histogram under these leaves.
hipError_t launch_equi_depth_leaves(const uint64_t* sorted_codes, uint64_t S, uint32_t L, uint32_t B,
                                    ModelHeader* hdr, const MlpState& ms, hipStream_t st);
// The MLP root's cell table over its L leaves (after training, the leaves and
// the choice of root; nothing is done unless the MLP root was chosen).
hipError_t launch_mlp_cell_table(const MlpState& ms, uint32_t L, const ModelHeader* hdr, hipStream_t st);
// Automatic kind: whether the linear root is kept (ModelHeader::mlp_skip);
// other kinds clear the flag.
hipError_t launch_auto_gate(const uint32_t* hist_rmi, uint32_t B, uint64_t S, float accept_ratio, uint32_t kind,
                            ModelHeader* hdr, hipStream_t st);
hipError_t launch_decide_root(const uint32_t* hist_rmi, const MlpState* ms, uint32_t B, uint64_t S,
                              float accept_ratio, uint32_t kind, ModelHeader* hdr, uint32_t* hist_used,
                              hipStream_t st);
// One training step on caller rows (verification): gradient, then the Adam
// update at step `step` (>= 1) of the FP32 parameters and moments, in place.
hipError_t launch_mlp_step(const MlpBlock* M, float* params, float* adam, const uint64_t* codes,
                           const float* targets, uint32_t step, float lr, float* grad, float* loss, hipStream_t st);
hipError_t mlp_prepare_kernels();
hipError_t launch_mlp_params_to_block(const float* d_params, const uint64_t* d_q9, MlpBlock* M, hipStream_t st);
hipError_t launch_mlp_eval(const MlpBlock* M, const uint64_t* codes, uint64_t n, float* y, hipStream_t st);
hipError_t launch_mlp_grad(const MlpBlock* M, const uint64_t* codes, const float* targets, float* grad,
                           float* loss, hipStream_t st);
constexpr uint32_t kMlpGradRows = 128;  // rows of one training step

// partition (k_partition.hip)
struct PassFilter {     // host tier: a chunk at input index idx_base, buckets lo .. hi-1 only
  uint64_t idx_base;
  uint32_t lo, hi;
};
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
hipError_t launch_partition(const ModelHeader* hdr, const Leaf* leaves, const MlpState* ms, const uint8_t* recs,
                            uint64_t n, uint32_t rec_bytes, uint32_t vk, uint8_t* part,
                            const PartLayout& lay, hipStream_t st, const PassFilter* filter = nullptr);
hipError_t launch_count(const ModelHeader* hdr, const Leaf* leaves, const MlpState* ms, const uint8_t* recs,
                        uint64_t n, uint32_t rec_bytes, uint32_t* counts, hipStream_t st, uint32_t vk = 0);
hipError_t launch_keys_differ(const uint8_t* recs, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                              const uint8_t* ref, uint32_t* flag, hipStream_t st);
hipError_t launch_exact_regions(const uint32_t* counts_all, uint32_t lo, uint32_t nb, uint64_t total, uint8_t* part,
                                const PartLayout& lay, hipStream_t st);
hipError_t launch_scan_counts(uint8_t* part, const PartLayout& lay, uint32_t B, uint64_t* offsets,
                              hipStream_t st);
hipError_t launch_spill_fixup(uint8_t* part, const PartLayout& lay, uint64_t n, hipStream_t st);

// bucket sort (k_bucket_sort.hip)
// key_bytes: bytes of the (virtual) key the composite holds, at most 12; vk
// as for virtual_key.
hipError_t launch_bucket_sort_small(uint8_t* part, const PartLayout& lay, uint32_t B, const uint64_t* offsets,
                                    uint32_t rec_bytes, uint32_t key_bytes, uint8_t* out, hipStream_t st,
                                    uint32_t vk = 0);
// whole jobs of up to kSmallCap records, one block each (batch)
struct TinyJob {
  const uint32_t* in;   // n records
  uint32_t* out;        // n records (may equal in)
  uint32_t n, pad;
  uint64_t staging_dw;  // dword offset of the job's staging copy (in-place jobs)
};
hipError_t launch_tiny_jobs(const TinyJob* d_jobs, uint32_t njobs, uint32_t rec_bytes, uint32_t key_bytes,
                            uint32_t* staging, hipStream_t st);
hipError_t launch_bucket_sort_large(uint8_t* part, const PartLayout& lay, uint32_t B, uint64_t n, const uint64_t* offsets,
                                    uint32_t rec_bytes, uint32_t key_bytes, uint8_t* out, hipStream_t st,
                                    uint32_t vk = 0);

// ---------------------------------------------------------- batch windows --
// A window of a batch: jobs whose sizes differ by at most 2x, whose partition
// buffers fit the window's workspace together, sorted by one launch per phase
// (capacities, partition, scan, spill fix-up, bucket sorts) instead of one
// launch per phase and job.  Every job of a window gets the same number G of
// blocks in a phase's grid: block b of the launch works for job b / G as its
// block b % G of G, so the mapping costs one division and no table.
struct WinJob {
  const uint8_t* recs;      // the job's records (device)
  uint8_t* out;             // its output, may equal recs
  uint64_t n, S;
  const ModelHeader* hdr;   // the job's fitted model
  const Leaf* leaves;       // RMI leaves
  const uint32_t* hist;     // sample keys per bucket under the root in use
  const MlpBlock* mlp;      // equi-depth roots only (else null): the network,
  const Leaf* eq_leaves;    // the equi-depth leaves and their routing tables
  const uint64_t* bound;
  const uint32_t* ccells;   // the spline root's code-cell table
  const uint32_t* cells;
  uint8_t* part;            // partition buffer laid out as lay
  uint64_t* offsets;        // B + 1 output offsets
  PartLayout lay;
  uint32_t B, pad_;
};
struct WinGrids {           // blocks per job of each phase's launch
  uint32_t part, fixup, small, mid, split, seg, gather;
};
// The grids of a window whose largest job has nmax records and B buckets at
// most; tiles_per_block: partition tiles per block (0: partition_grid's rule).
WinGrids window_grids(uint64_t nmax, uint32_t Bmax, uint32_t tiles_per_block);
uint32_t partition_grid(uint64_t n);    // blocks of the partition of n records
uint32_t spill_fixup_grid(uint64_t n);  // blocks of the spill fix-up of n records
hipError_t launch_capacities_win(const WinJob* jobs, uint32_t njobs, uint32_t region_pct, hipStream_t st);
hipError_t launch_partition_win(const WinJob* jobs, uint32_t njobs, uint32_t G, uint32_t rec_bytes, bool equi_depth,
                                hipStream_t st);
hipError_t launch_scan_counts_win(const WinJob* jobs, uint32_t njobs, hipStream_t st);
hipError_t launch_spill_fixup_win(const WinJob* jobs, uint32_t njobs, uint32_t G, hipStream_t st);
hipError_t launch_bucket_sort_small_win(const WinJob* jobs, uint32_t njobs, uint32_t G, uint32_t rec_bytes,
                                        uint32_t key_bytes, hipStream_t st);
hipError_t launch_bucket_sort_large_win(const WinJob* jobs, uint32_t njobs, const WinGrids& g, uint32_t rec_bytes,
                                        uint32_t key_bytes, hipStream_t st);

}  // namespace elsar
