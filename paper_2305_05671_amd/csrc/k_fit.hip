// Sample, sample sort and RMI fit kernels (gfx950).
//
// Training sample (Section 3.1): S = min(max(ceil(n/100), 1024), 1e7, n) keys,
// sample s drawn uniformly from the stratum [floor(s*n/S), floor((s+1)*n/S))
// by a Philox4x32-10 draw keyed by the seed.  The sample's base-95 codes
// (Section 4) are radix-sorted on the device; their ranks are the empirical
// CDF the two-level RMI (Section 3.1) is fitted to.
#include "elsar_internal.h"

namespace elsar {

// ------------------------------------------------------------- sampling --
// Record of sample s: uniform (one Philox draw) within the stratum
// [floor(s n / S), floor((s+1) n / S)).
__device__ __forceinline__ uint64_t sample_index(uint64_t s, uint64_t n, uint64_t S, uint64_t seed) {
  const uint64_t lo = s * n / S, hi = (s + 1) * n / S;
  const uint32_t u = philox_x(s, 0x53414D50u, 0u, seed);
  return lo + (((uint64_t)u * (hi - lo)) >> 32);
}

__global__ __launch_bounds__(256) void sample_codes_kernel(const uint8_t* __restrict__ recs, uint64_t n,
                                                           uint32_t rec_bytes, uint64_t S, uint64_t seed,
                                                           uint64_t* __restrict__ codes, uint32_t vk) {
  uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (s >= S) return;
  const uint32_t* r = reinterpret_cast<const uint32_t*>(recs + sample_index(s, n, S, seed) * rec_bytes);
  uint32_t r0 = r[0], r1 = r[1], r2 = vk ? r[2] : 0u;
  virtual_key(r0, r1, r2, vk);
  codes[s] = key_code(r0, r1);
}

hipError_t launch_sample_codes(const uint8_t* recs, uint64_t n, uint32_t rec_bytes, uint64_t S, uint64_t seed,
                               uint64_t* codes, hipStream_t st, uint32_t vk) {
  if (S == 0) return hipSuccess;
  uint32_t grid = (uint32_t)((S + 255) / 256);
  sample_codes_kernel<<<grid, 256, 0, st>>>(recs, n, rec_bytes, S, seed, codes, vk);
  return hipGetLastError();
}

// ---------------------------------------------- LSD radix sort of u64 keys --
// Per pass (one byte): per-tile digit histograms (digit-major), one exclusive
// scan over them, then a stable scatter where each wave ranks its own items in
// order with ballot-matched digits.  With few tiles (a sample of up to 64K
// codes) the scatter blocks scan the counts themselves and the scan kernel's
// launch is saved: at 10^4 codes a pass costs launches, not bandwidth.
constexpr int kRadixThreads = 256;
constexpr int kRadixRounds = 16;  // rounds of 64 items per wave
constexpr int kRadixWaves = kRadixThreads / 64;
constexpr int kRadixTile = kRadixThreads * kRadixRounds;  // 4096
constexpr uint32_t kRadixFuseTiles = 16;  // up to this many tiles the scatter scans the tile counts itself

__global__ __launch_bounds__(kRadixThreads) void radix_hist_kernel(const uint64_t* __restrict__ keys, uint64_t n,
                                                                   int shift, uint32_t ntiles,
                                                                   uint32_t* __restrict__ tile_hist) {
  __shared__ uint32_t cnt[256];
  cnt[threadIdx.x] = 0;
  const uint64_t base = (uint64_t)blockIdx.x * kRadixTile;
  // every load first, unconditionally (the index clamped to the last key):
  // a load under "i < n" was waited for inside its branch, one round trip
  // per key
  uint64_t key[kRadixRounds];
#pragma unroll
  for (int k = 0; k < kRadixRounds; ++k) {
    const uint64_t i = base + (uint64_t)k * kRadixThreads + threadIdx.x;
    key[k] = keys[i < n ? i : n - 1];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kRadixRounds; ++k) {
    const uint64_t i = base + (uint64_t)k * kRadixThreads + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(key[k] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  tile_hist[(uint64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Per digit d (one block each): exclusive scan over the tiles of d's counts,
// in place; digit_tot[d] gets d's total.
__global__ __launch_bounds__(256) void radix_digit_scan_kernel(uint32_t* __restrict__ tile_hist, uint32_t ntiles,
                                                               uint32_t* __restrict__ digit_tot) {
  __shared__ uint32_t sh[256 / 64 + 1];
  uint32_t* v = tile_hist + (uint64_t)blockIdx.x * ntiles;
  uint32_t carry = 0;
  for (uint32_t base = 0; base < ntiles; base += 256 * 4) {
    uint32_t c[4], s = 0;
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
      uint32_t t = base + threadIdx.x * 4 + i;
      c[i] = t < ntiles ? v[t] : 0u;
      s += c[i];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan<uint32_t, 256>(s, sh, &tot);
#pragma unroll
    for (uint32_t i = 0; i < 4; ++i) {
      uint32_t t = base + threadIdx.x * 4 + i;
      if (t < ntiles) v[t] = run;
      run += c[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

// fused (few tiles): tile_off holds the raw per-tile counts and digit_tot is
// unused; each block sums, per digit, all tiles and the tiles before its own,
// which replaces the digit-scan launch.
__global__ __launch_bounds__(kRadixThreads) void radix_scatter_kernel(const uint64_t* __restrict__ in,
                                                                      uint64_t* __restrict__ out, uint64_t n,
                                                                      int shift, uint32_t ntiles,
                                                                      const uint32_t* __restrict__ tile_off,
                                                                      const uint32_t* __restrict__ digit_tot,
                                                                      bool fused) {
  __shared__ uint32_t wc[kRadixWaves][256];
  __shared__ uint32_t gbase[256];
  __shared__ uint32_t sh[kRadixThreads / 64 + 1];
  const uint32_t w = threadIdx.x >> 6;
  for (uint32_t i = threadIdx.x; i < kRadixWaves * 256; i += kRadixThreads) (&wc[0][0])[i] = 0;
  __syncthreads();
  uint64_t base = (uint64_t)blockIdx.x * kRadixTile + (uint64_t)w * 64 * kRadixRounds;
  uint64_t key[kRadixRounds];
  uint32_t loc[kRadixRounds];
  // every load first, the tile's digit offsets included (the key index
  // clamped to the last key; invalid lanes take no part below): issued
  // inside the rank loop, each round's load was waited for before the next
  // one went out
#pragma unroll
  for (int r = 0; r < kRadixRounds; ++r) {
    const uint64_t i = base + (uint64_t)r * 64 + lane_id();
    key[r] = in[i < n ? i : n - 1];
  }
  uint32_t dtot, before = 0, total = 0;
  if (fused) {
    const uint32_t* h = tile_off + (uint64_t)threadIdx.x * ntiles;
    for (uint32_t t = 0; t < ntiles; ++t) {
      const uint32_t c = h[t];
      before += t < blockIdx.x ? c : 0u;
      total += c;
    }
  } else {
    before = tile_off[(uint64_t)threadIdx.x * ntiles + blockIdx.x];
    total = digit_tot[threadIdx.x];
  }
#pragma unroll
  for (int r = 0; r < kRadixRounds; ++r) {
    uint64_t i = base + (uint64_t)r * 64 + lane_id();
    bool valid = i < n;
    uint32_t d = (uint32_t)(key[r] >> shift) & 0xFFu;
    uint64_t peers = match_digit8(d, valid);
    uint32_t rank = __popcll(peers & lanemask_lt());
    uint32_t prev = valid ? wc[w][d] : 0u;
    loc[r] = prev + rank;
    __builtin_amdgcn_wave_barrier();
    if (valid && rank == 0) wc[w][d] = prev + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  uint32_t dbase = block_exclusive_scan<uint32_t, kRadixThreads>(total, sh, &dtot);
  {
    uint32_t d = threadIdx.x, run = 0;
    for (int ww = 0; ww < kRadixWaves; ++ww) {
      uint32_t c = wc[ww][d];
      wc[ww][d] = run;
      run += c;
    }
    gbase[d] = dbase + before;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRadixRounds; ++r) {
    uint64_t i = base + (uint64_t)r * 64 + lane_id();
    if (i < n) {
      uint32_t d = (uint32_t)(key[r] >> shift) & 0xFFu;
      out[(uint64_t)gbase[d] + wc[w][d] + loc[r]] = key[r];
    }
  }
}

size_t radix_u64_scratch_bytes(uint64_t n) {
  uint64_t ntiles = (n + kRadixTile - 1) / kRadixTile;
  return (size_t)((ntiles + 1) * 256 * sizeof(uint32_t));
}

// Sort bytes lo_byte..hi_byte (inclusive) of keys; *sorted = buffer with the result.
hipError_t launch_radix_sort_u64(uint64_t* keys, uint64_t* tmp, uint64_t n, int lo_byte, int hi_byte,
                                 void* scratch, hipStream_t st, uint64_t** sorted) {
  *sorted = keys;
  if (n <= 1) return hipSuccess;
  uint32_t ntiles = (uint32_t)((n + kRadixTile - 1) / kRadixTile);
  uint32_t* th = static_cast<uint32_t*>(scratch);
  uint32_t* dtot = th + (uint64_t)ntiles * 256;
  uint64_t *a = keys, *b = tmp;
  for (int byte = lo_byte; byte <= hi_byte; ++byte) {
    int shift = 8 * byte;
    const bool fused = ntiles <= kRadixFuseTiles;
    radix_hist_kernel<<<ntiles, kRadixThreads, 0, st>>>(a, n, shift, ntiles, th);
    if (!fused) radix_digit_scan_kernel<<<256, 256, 0, st>>>(th, ntiles, dtot);
    radix_scatter_kernel<<<ntiles, kRadixThreads, 0, st>>>(a, b, n, shift, ntiles, th, dtot, fused);
    uint64_t* t = a;
    a = b;
    b = t;
  }
  *sorted = a;
  return hipGetLastError();
}

// ------------------------------------------------------------ RMI fitting --
// Root: least squares (FP64, centred two-pass) of t = L*s/S on x = f32(code_s).
// Deterministic: fixed block decomposition and fixed reduction trees.
constexpr int kFitThreads = 256;
constexpr int kFitBlocks = 256;

__device__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kFitThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kFitThreads) void root_sum_x_kernel(const uint64_t* __restrict__ e, uint64_t S,
                                                                 double* __restrict__ part_x) {
  __shared__ double sh[kFitThreads];
  double sx = 0;
  for (uint64_t s = blockIdx.x * (uint64_t)kFitThreads + threadIdx.x; s < S; s += (uint64_t)kFitBlocks * kFitThreads)
    sx += (double)code_f32(e[s]);
  double t = block_sum(sx, sh);
  if (threadIdx.x == 0) part_x[blockIdx.x] = t;
}

__global__ __launch_bounds__(kFitThreads) void root_moments_kernel(const uint64_t* __restrict__ e, uint64_t S,
                                                                   uint32_t L, const double* __restrict__ part_x,
                                                                   double* __restrict__ part_xx,
                                                                   double* __restrict__ part_xt) {
  __shared__ double sh[kFitThreads];
  double mx = block_sum(part_x[threadIdx.x], sh) / (double)S;  // kFitBlocks == kFitThreads
  double mt = (double)L * (double)(S - 1) / (2.0 * (double)S);
  double sxx = 0, sxt = 0;
  for (uint64_t s = blockIdx.x * (uint64_t)kFitThreads + threadIdx.x; s < S;
       s += (uint64_t)kFitBlocks * kFitThreads) {
    double dx = (double)code_f32(e[s]) - mx;
    double dt = (double)L * (double)s / (double)S - mt;
    sxx += dx * dx;
    sxt += dx * dt;
  }
  double a = block_sum(sxx, sh);
  double b = block_sum(sxt, sh);
  if (threadIdx.x == 0) {
    part_xx[blockIdx.x] = a;
    part_xt[blockIdx.x] = b;
  }
}

// Least-squares line of t = L*s/S on x (centred sums), slope clamped at 0.
__device__ __forceinline__ void root_line(double mx, double sxx, double sxt, uint32_t L, uint64_t S, double* a0,
                                          double* a1) {
  const double mt = (double)L * (double)(S - 1) / (2.0 * (double)S);
  double b = sxx > 0 ? sxt / sxx : 0.0;
  if (b < 0) {
    *a1 = 0;
    *a0 = mt;
  } else {
    *a1 = b;
    *a0 = mt - b * mx;
  }
}

__global__ __launch_bounds__(kFitThreads) void root_final_kernel(uint64_t S, uint64_t n, uint32_t L, uint32_t B,
                                                                 const double* __restrict__ part_x,
                                                                 const double* __restrict__ part_xx,
                                                                 const double* __restrict__ part_xt,
                                                                 ModelHeader* __restrict__ hdr) {
  __shared__ double sh[kFitThreads];
  double mx = block_sum(part_x[threadIdx.x], sh) / (double)S;
  double sxx = block_sum(part_xx[threadIdx.x], sh);
  double sxt = block_sum(part_xt[threadIdx.x], sh);
  if (threadIdx.x == 0) {
    double a0, a1;
    root_line(mx, sxx, sxt, L, S, &a0, &a1);
    hdr->a0 = (float)a0;
    hdr->a1 = (float)a1;
    hdr->L = L;
    hdr->B = B;
    hdr->kind_used = 0;
    hdr->mlp_rejected = 0;
    hdr->n_fit = n;
    hdr->S = S;
    hdr->max_sample_run = 0;
    hdr->mlp_L = 0;
    hdr->mlp_skip = 0;
    hdr->max_rmi = hdr->max_eq = hdr->max_net = hdr->rmi_ok = 0;
    hdr->perfect = 0.0f;
  }
}

// Leaf j: samples f..g-1 routed to it by the root (contiguous: routing is
// monotone).  Linear spline from (0, B*f/S) to (x(e[g-1]-e[f]), B*(g-1)/S);
// bucket range [B*f/S, min(B*(g-1)/S, B-1)].  Empty leaves are constant at the
// next non-empty leaf's first bucket.
__device__ uint64_t first_in_leaf(const uint64_t* e, uint64_t S, float a0, float a1, uint32_t L, uint32_t j) {
  uint64_t lo = 0, hi = S;
  while (lo < hi) {
    uint64_t mid = lo + ((hi - lo) >> 1);
    if (rmi_leaf(a0, a1, L, e[mid]) < j) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ Leaf spline_leaf(const uint64_t* e, uint64_t S, uint32_t B, uint64_t f, uint64_t g) {
  Leaf lf;
  lf.pad[0] = lf.pad[1] = 0;
  if (f == g) {
    uint32_t v = f < S ? (uint32_t)(((uint64_t)B * f) / S) : B - 1;
    lf.base = 0;
    lf.c = 0.0f;
    lf.b = (float)v;
    lf.lo = lf.hi = v;
  } else {
    double tf = (double)B * (double)f / (double)S;
    double tl = (double)B * (double)(g - 1) / (double)S;
    double span = (double)code_f32(e[g - 1] - e[f]);
    double cj = span > 0 ? (tl - tf) / span : 0.0;
    lf.base = e[f];
    lf.c = (float)cj;
    lf.b = (float)tf;
    lf.lo = (uint32_t)(((uint64_t)B * f) / S);
    uint64_t h = ((uint64_t)B * (g - 1)) / S;
    lf.hi = (uint32_t)(h < B - 1 ? h : B - 1);
  }
  return lf;
}

__global__ __launch_bounds__(256) void leaf_fit_kernel(const uint64_t* __restrict__ e, uint64_t S,
                                                       const ModelHeader* __restrict__ hdr,
                                                       Leaf* __restrict__ leaves) {
  uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t L = hdr->L, B = hdr->B;
  if (j >= L) return;
  const float a0 = hdr->a0, a1 = hdr->a1;
  uint64_t f = first_in_leaf(e, S, a0, a1, L, j);
  uint64_t g = j + 1 < L ? first_in_leaf(e, S, a0, a1, L, j + 1) : S;
  leaves[j] = spline_leaf(e, S, B, f, g);
}

size_t fit_scratch_bytes(uint64_t /*S*/) { return 3 * kFitBlocks * sizeof(double); }

hipError_t launch_fit_rmi(const uint64_t* e, uint64_t S, uint64_t n, uint32_t L, uint32_t B, ModelHeader* hdr,
                          Leaf* leaves, void* scratch, hipStream_t st) {
  double* px = static_cast<double*>(scratch);
  double* pxx = px + kFitBlocks;
  double* pxt = pxx + kFitBlocks;
  root_sum_x_kernel<<<kFitBlocks, kFitThreads, 0, st>>>(e, S, px);
  root_moments_kernel<<<kFitBlocks, kFitThreads, 0, st>>>(e, S, L, px, pxx, pxt);
  root_final_kernel<<<1, kFitThreads, 0, st>>>(S, n, L, B, px, pxx, pxt, hdr);
  leaf_fit_kernel<<<(L + 255) / 256, 256, 0, st>>>(e, S, hdr, leaves);
  return hipGetLastError();
}

// -------------------------------------------------------- bucket capacity --
// h_j = sample keys the fitted model puts in bucket j.  The partition reserves
// ceil(f * max(n * (h_j + 2 sqrt(h_j)) / S, n / B)) + 16 slots for bucket j
// (f = region_pct/100, default 1.25), rounded up to even; records beyond
// continue in the spill.
// Sample keys per bucket.  The sample is usually sorted, so neighbouring lanes
// share buckets: one atomic per run of equal buckets within the wave.
__global__ __launch_bounds__(256) void sample_bucket_hist_kernel(const uint64_t* __restrict__ e, uint64_t S,
                                                                 const ModelHeader* __restrict__ hdr,
                                                                 const Leaf* __restrict__ leaves,
                                                                 uint32_t* __restrict__ hist) {
  const uint64_t s = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  const bool in = s < S;
  const uint64_t c = e[in ? s : S - 1];
  const uint32_t b = leaf_bucket(load_leaf(leaves, rmi_leaf(hdr->a0, hdr->a1, hdr->L, c)), c);
  const uint32_t l = __lane_id();
  const uint32_t bl = __shfl_up(b, 1), br = __shfl_down(b, 1);
  const bool start = in && (l == 0 || bl != b);
  const bool last = in && (l == 63 || br != b || s + 1 == S);
  const uint64_t starts = __ballot(start);
  if (last) {
    const uint64_t below = starts & (l == 63 ? ~0ull : ((2ull << l) - 1));  // starts at lanes <= l
    const uint32_t first_lane = 63u - (uint32_t)__clzll((long long)below);
    atomicAdd(&hist[b], l + 1 - first_lane);
  }
}

// A plain fill: it records as a kernel node under graph capture, which a
// memset does not do reliably.
__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint64_t n, uint32_t v) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  fill_u32_kernel<<<(uint32_t)(blocks < 1024 ? blocks : 1024), 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_sample_hist(const ModelHeader* hdr, const Leaf* leaves, const uint64_t* e, uint64_t S,
                              uint32_t B, uint32_t* hist, hipStream_t st) {
  hipError_t err = launch_fill_u32(hist, B, 0u, st);
  if (err != hipSuccess) return err;
  if (S) sample_bucket_hist_kernel<<<(uint32_t)((S + 255) / 256), 256, 0, st>>>(e, S, hdr, leaves, hist);
  return hipGetLastError();
}

// ---------------------------------------------- radix (equi-width) model --
// No learned model: the root sends every code to leaf 0 (a0 = a1 = 0), whose
// line maps the whole code range [0, 95^8) linearly onto the B buckets.
__global__ void radix_model_kernel(uint64_t S, uint64_t n, uint32_t L, uint32_t B, ModelHeader* __restrict__ hdr,
                                   Leaf* __restrict__ leaves) {
  for (uint32_t j = threadIdx.x; j < L; j += blockDim.x) {
    Leaf lf;
    lf.base = 0;
    lf.c = (float)((double)B / 6634204312890625.0);  // 95^8
    lf.b = 0.0f;
    lf.lo = 0;
    lf.hi = B - 1;
    lf.pad[0] = lf.pad[1] = 0;
    leaves[j] = lf;
  }
  if (threadIdx.x == 0) {
    hdr->a0 = 0.0f;
    hdr->a1 = 0.0f;
    hdr->L = L;
    hdr->B = B;
    hdr->kind_used = 0;
    hdr->mlp_rejected = 0;
    hdr->n_fit = n;
    hdr->S = S;
    hdr->max_sample_run = 0;
    hdr->mlp_L = 0;
    hdr->mlp_skip = 0;
    hdr->max_rmi = hdr->max_eq = hdr->max_net = hdr->rmi_ok = 0;
    hdr->perfect = 0.0f;
  }
}

hipError_t launch_radix_model(uint64_t S, uint64_t n, uint32_t L, uint32_t B, ModelHeader* hdr, Leaf* leaves,
                              hipStream_t st) {
  radix_model_kernel<<<1, 256, 0, st>>>(S, n, L, B, hdr, leaves);
  return hipGetLastError();
}

// ---------------------------------------------------- batch: fit per job --
// One 1024-thread block fits the whole model of one job: its S sample codes
// are drawn straight from the job's records and sorted, then the root line,
// the spline leaves and the sample histogram are computed as by the per-job
// kernels.  A sample of up to kBatchFitMaxS codes is sorted in LDS (bitonic
// network) and read there; a larger one (up to kBatchFitChunks chunks of
// kBatchFitMaxS) is sorted chunk by chunk in LDS into the job's global
// scratch, the sorted chunks are merged by rank into its second half, and the
// fit reads that (a few hundred KB, held in L2).
constexpr uint32_t kBfThreads = 1024;

__device__ double bf_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  for (uint32_t i = 0; i < kBfThreads / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// Sample codes c0 .. c0+m-1 of job J sorted into e[0 .. m) (LDS); the
// bitonic network runs over the next power of two, padded with codes that
// sort last.
__device__ __forceinline__ void bf_sort_chunk(const FitJob& J, uint32_t rec_bytes, uint64_t c0, uint32_t m,
                                              uint64_t* e) {
  const uint32_t tid = threadIdx.x;
  uint32_t P = 1;
  while (P < m) P <<= 1;
  for (uint32_t s = tid; s < P; s += kBfThreads) {
    uint64_t c = ~0ull;
    if (s < m) {
      const uint32_t* r =
          reinterpret_cast<const uint32_t*>(J.recs + sample_index(c0 + s, J.n, J.S, J.seed) * rec_bytes);
      c = key_code(r[0], r[1]);
    }
    e[s] = c;
  }
  __syncthreads();
  for (uint32_t k = 2; k <= P; k <<= 1)
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = tid; i < P; i += kBfThreads) {
        const uint32_t ij = i ^ j;
        if (ij > i) {
          const uint64_t a = e[i], b = e[ij];
          if ((a > b) == ((i & k) == 0)) {
            e[i] = b;
            e[ij] = a;
          }
        }
      }
      __syncthreads();
    }
}

// Codes of the sorted run g[0 .. len) below x (or, with upper, not above x).
__device__ __forceinline__ uint32_t bf_rank(const uint64_t* g, uint32_t len, uint64_t x, bool upper) {
  uint32_t lo = 0, hi = len;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    const uint64_t v = g[mid];
    if (v < x || (upper && v == x)) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The model from the sorted sample e[0 .. S) (LDS or global).
__device__ __forceinline__ void bf_fit_sorted(const FitJob& J, const uint64_t* e, double* sh, uint32_t* shm) {
  const uint32_t tid = threadIdx.x;
  {
    const uint64_t S = J.S;
    // root line
    double sx = 0;
    for (uint32_t s = tid; s < S; s += kBfThreads) sx += (double)code_f32(e[s]);
    const double mx = bf_sum(sx, sh) / (double)S;
    const double mt = (double)J.L * (double)(S - 1) / (2.0 * (double)S);
    double sxx = 0, sxt = 0;
    for (uint32_t s = tid; s < S; s += kBfThreads) {
      const double dx = (double)code_f32(e[s]) - mx;
      const double dt = (double)J.L * (double)s / (double)S - mt;
      sxx += dx * dx;
      sxt += dx * dt;
    }
    sxx = bf_sum(sxx, sh);
    sxt = bf_sum(sxt, sh);
    double a0d, a1d;
    root_line(mx, sxx, sxt, J.L, S, &a0d, &a1d);
    const float a0 = (float)a0d, a1 = (float)a1d;
    // leaves, then the histogram of the sample over the buckets
    for (uint32_t j = tid; j < J.L; j += kBfThreads) {
      const uint64_t f = first_in_leaf(e, S, a0, a1, J.L, j);
      const uint64_t g = j + 1 < J.L ? first_in_leaf(e, S, a0, a1, J.L, j + 1) : S;
      J.leaves[j] = spline_leaf(e, S, J.B, f, g);
    }
    for (uint32_t b = tid; b < J.B; b += kBfThreads) J.hist[b] = 0;
    __syncthreads();
    for (uint32_t s = tid; s < S; s += kBfThreads)
      atomicAdd(&J.hist[leaf_bucket(load_leaf(J.leaves, rmi_leaf(a0, a1, J.L, e[s])), e[s])], 1u);
    __syncthreads();
    uint32_t m = 0;
    for (uint32_t b = tid; b < J.B; b += kBfThreads) m = J.hist[b] > m ? J.hist[b] : m;
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t o = __shfl_xor(m, off);
      m = o > m ? o : m;
    }
    if (lane_id() == 0) shm[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
      uint32_t mm = 0;
      for (uint32_t i = 0; i < kBfThreads / 64; ++i) mm = shm[i] > mm ? shm[i] : mm;
      ModelHeader* h = J.hdr;
      h->a0 = a0;
      h->a1 = a1;
      h->L = J.L;
      h->B = J.B;
      h->kind_used = 0;
      h->mlp_rejected = 0;
      h->n_fit = J.n;
      h->S = S;
      h->max_sample_bucket = mm;
      h->opt_sample_bucket = (uint32_t)((S + J.B - 1) / J.B);
      h->max_sample_run = 0;
      h->mlp_L = 0;
      h->mlp_skip = 0;
      h->max_rmi = mm;
      h->max_eq = h->max_net = h->rmi_ok = 0;
      h->perfect = 0.0f;
    }
    __syncthreads();
  }
}

__device__ void fit_job_block(const FitJob& J, uint32_t rec_bytes, uint64_t* e, double* sh, uint32_t* shm) {
  const uint64_t S = J.S;
  if (S <= kBatchFitMaxS) {
    bf_sort_chunk(J, rec_bytes, 0, (uint32_t)S, e);
    bf_fit_sorted(J, e, sh, shm);
    return;
  }
  // chunks sorted in LDS into g, merged by rank into g2: a code at index i of
  // chunk a goes to i + (codes not above it in earlier chunks) + (codes below
  // it in later chunks), a permutation that orders the whole sample
  uint64_t* g = J.scratch;
  uint64_t* g2 = J.scratch + S;
  const uint32_t nc = (uint32_t)((S + kBatchFitMaxS - 1) / kBatchFitMaxS);
  for (uint32_t a = 0; a < nc; ++a) {
    const uint64_t c0 = (uint64_t)a * kBatchFitMaxS;
    const uint32_t m = (uint32_t)(S - c0 < kBatchFitMaxS ? S - c0 : kBatchFitMaxS);
    bf_sort_chunk(J, rec_bytes, c0, m, e);
    for (uint32_t i = threadIdx.x; i < m; i += kBfThreads) g[c0 + i] = e[i];
    __syncthreads();
  }
  for (uint32_t s = threadIdx.x; s < S; s += kBfThreads) {
    const uint32_t a = s / kBatchFitMaxS;
    const uint64_t x = g[s];
    uint64_t pos = s - (uint64_t)a * kBatchFitMaxS;
    for (uint32_t b = 0; b < nc; ++b) {
      if (b == a) continue;
      const uint64_t b0 = (uint64_t)b * kBatchFitMaxS;
      const uint32_t len = (uint32_t)(S - b0 < kBatchFitMaxS ? S - b0 : kBatchFitMaxS);
      pos += bf_rank(g + b0, len, x, b < a);
    }
    g2[pos] = x;
  }
  __syncthreads();
  bf_fit_sorted(J, g2, sh, shm);
}

__global__ __launch_bounds__(kBfThreads) void batch_fit_kernel(const FitJob* __restrict__ jobs, uint32_t njobs,
                                                               uint32_t rec_bytes) {
  __shared__ uint64_t e[kBatchFitMaxS];
  __shared__ double sh[kBfThreads / 64];
  __shared__ uint32_t shm[kBfThreads / 64];
  for (uint32_t jb = blockIdx.x; jb < njobs; jb += gridDim.x) fit_job_block(jobs[jb], rec_bytes, e, sh, shm);
}


hipError_t launch_batch_fit(const FitJob* d_jobs, uint32_t njobs, uint32_t rec_bytes, hipStream_t st) {
  if (njobs == 0) return hipSuccess;
  batch_fit_kernel<<<njobs < 2048 ? njobs : 2048, kBfThreads, 0, st>>>(d_jobs, njobs, rec_bytes);
  return hipGetLastError();
}

constexpr uint32_t kScanThreads = 1024;

// Region sizes and starts, in one block.  Wave w owns a contiguous segment of
// WS buckets (WS a multiple of 1024) and walks it 256 buckets a step, lane l
// taking buckets 4l .. 4l+3 of the step with 16-byte loads and stores, so
// that every access of a wave covers whole lines (one segment per thread made
// each access touch 64 lines, all through the one CU).  The loads of four
// steps are issued before any is used.  Pass 1 sums the wave's sizes; the
// waves' sums are scanned in order; pass 2 recomputes the sizes, scans them
// across the wave step by step and writes sizes, starts and cleared fill
// counters.  A region past the reserved slot count cannot happen by
// construction; such a bucket would get no region and all its records would
// spill.
constexpr uint32_t kScanWaves = kScanThreads / 64;

// Region size of a bucket with h sample keys: they estimate its mass as h / S
// with a standard deviation of about sqrt(h) / S, and the region covers two of
// them beyond the estimate, at least the ideal n / B, times the slack factor
// (the root in single precision: h is exact there, and FP64 square roots and
// divisions took most of the one-block kernel's time).  per = n / S.
__device__ __forceinline__ uint32_t region_slots(uint32_t h, double per, double ideal, double scale) {
  const double hd = (double)h;
  const double expect = (hd + 2.0 * (double)sqrtf((float)h)) * per;
  const double m = expect > ideal ? expect : ideal;
  return ((uint32_t)ceil(scale * m) + 16u + 1u) & ~1u;
}

__device__ __forceinline__ void init_part_header(PartHeader* ph, uint64_t n, uint64_t cap_slots, uint32_t B) {
  ph->n = n;
  ph->cap_slots = cap_slots;
  ph->B = B;
  ph->spill_count = 0;
  ph->n_mid = 0;
  ph->n_mid_hi = 0;
  ph->n_big = 0;
  ph->n_big2 = 0;
  ph->max_count = 0;
  ph->mid_records = 0;
  ph->big_records = 0;
}

constexpr uint32_t kCapSteps = 8;  // steps of 256 buckets whose sample counts are loaded together

__device__ __forceinline__ void capacity_body(const uint32_t* __restrict__ hist, uint64_t S, uint64_t n, uint32_t B,
                                              double scale, uint32_t* __restrict__ caps,
                                              uint32_t* __restrict__ rstart, uint32_t* __restrict__ counts,
                                              uint32_t cstride, PartHeader* __restrict__ ph, uint64_t cap_slots) {
  __shared__ uint64_t sh[kScanWaves];
  const double ideal = (double)n / (double)B;
  const uint32_t WS = ((B + kScanWaves - 1) / kScanWaves + 1023) & ~1023u;
  const uint32_t w = threadIdx.x >> 6, l = lane_id();
  const uint32_t s0 = w * WS, s1 = s0 + WS < B ? s0 + WS : B;  // empty when s0 >= B
  // sample counts of buckets j .. j+3 (zero past the segment), one 16-byte
  // load with no branch around it (a load inside a branch is waited for
  // there, which made the steps' loads one round trip each): past the end of
  // the histogram it reads its last vector again, and the histogram's space,
  // rounded up to a multiple of 256 bytes, keeps that vector's tail in bounds
  const uint32_t jlast = (B - 1) & ~3u;
  auto load4 = [&](uint32_t j, uint32_t h[4]) {
    const uint4 x = *reinterpret_cast<const uint4*>(hist + (j < B ? j : jlast));
    h[0] = j < s1 ? x.x : 0u;
    h[1] = j + 1 < s1 ? x.y : 0u;
    h[2] = j + 2 < s1 ? x.z : 0u;
    h[3] = j + 3 < s1 ? x.w : 0u;
  };
  const double per = (double)n / (double)S;
  auto size_of = [&](uint32_t j, uint32_t h) { return j < s1 ? region_slots(h, per, ideal, scale) : 0u; };
  uint64_t s = 0;
  for (uint32_t jb = s0; jb < s1; jb += 256 * kCapSteps) {
    uint32_t h[kCapSteps][4];
#pragma unroll
    for (uint32_t u = 0; u < kCapSteps; ++u) load4(jb + 256 * u + 4 * l, h[u]);
#pragma unroll
    for (uint32_t u = 0; u < kCapSteps; ++u)
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) s += size_of(jb + 256 * u + 4 * l + q, h[u][q]);
  }
  for (int off = 32; off >= 1; off >>= 1) s += shfl_xor_u64(s, off);
  if (l == 0) sh[w] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t r = 0;
    for (uint32_t i = 0; i < kScanWaves; ++i) {
      const uint64_t c = sh[i];
      sh[i] = r;
      r += c;
    }
  }
  __syncthreads();
  uint64_t run = sh[w];
  for (uint32_t jb = s0; jb < s1; jb += 256 * kCapSteps) {
    uint32_t h[kCapSteps][4];
#pragma unroll
    for (uint32_t u = 0; u < kCapSteps; ++u) load4(jb + 256 * u + 4 * l, h[u]);
#pragma unroll
    for (uint32_t u = 0; u < kCapSteps; ++u) {
      const uint32_t j = jb + 256 * u + 4 * l;
      uint32_t c[4];
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) c[q] = size_of(j + q, h[u][q]);
      const uint64_t own = (uint64_t)c[0] + c[1] + c[2] + c[3];
      const uint64_t x = wave_inclusive_scan<uint64_t>(own);
      uint64_t r = run + x - own;
      uint32_t cp[4], rp[4];
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const bool fits = r + c[q] <= cap_slots;
        cp[q] = fits ? c[q] : 0u;
        rp[q] = fits ? (uint32_t)r : 0u;
        r += c[q];
      }
      if (j + 4 <= s1) {
        *reinterpret_cast<uint4*>(caps + j) = make_uint4(cp[0], cp[1], cp[2], cp[3]);
        *reinterpret_cast<uint4*>(rstart + j) = make_uint4(rp[0], rp[1], rp[2], rp[3]);
        if (cstride == 1) {
          *reinterpret_cast<uint4*>(counts + j) = make_uint4(0, 0, 0, 0);
        } else {
#pragma unroll
          for (uint32_t q = 0; q < 4; ++q) counts[(uint64_t)(j + q) * cstride] = 0;
        }
      } else {
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
          if (j + q < s1) {
            caps[j + q] = cp[q];
            rstart[j + q] = rp[q];
            counts[(uint64_t)(j + q) * cstride] = 0;
          }
        }
      }
      run += shfl_u64(x, 63);  // the step's sum
    }
  }
  if (threadIdx.x == 0) init_part_header(ph, n, cap_slots, B);
}

__global__ __launch_bounds__(kScanThreads) void capacity_kernel(const uint32_t* __restrict__ hist, uint64_t S,
                                                                uint64_t n, uint32_t B, double scale,
                                                                uint32_t* __restrict__ caps,
                                                                uint32_t* __restrict__ rstart,
                                                                uint32_t* __restrict__ counts, uint32_t cstride,
                                                                PartHeader* __restrict__ ph, uint64_t cap_slots) {
  capacity_body(hist, S, n, B, scale, caps, rstart, counts, cstride, ph, cap_slots);
}

// A window of a batch: one block per job.
__global__ __launch_bounds__(kScanThreads) void capacity_win_kernel(const WinJob* __restrict__ jobs, double scale) {
  const WinJob& J = jobs[blockIdx.x];
  uint8_t* part = J.part;
  capacity_body(J.hist, J.S, J.n, J.B, scale, reinterpret_cast<uint32_t*>(part + J.lay.caps),
                reinterpret_cast<uint32_t*>(part + J.lay.rstart), reinterpret_cast<uint32_t*>(part + J.lay.pcounts),
                J.lay.cstride, reinterpret_cast<PartHeader*>(part + J.lay.header), J.lay.cap_slots);
}

hipError_t launch_capacities_win(const WinJob* jobs, uint32_t njobs, uint32_t region_pct, hipStream_t st) {
  if (njobs == 0) return hipSuccess;
  capacity_win_kernel<<<njobs, kScanThreads, 0, st>>>(jobs, region_pct / 100.0);
  return hipGetLastError();
}

// Many buckets: the same sizes and starts in two launches over chunks of
// kScanChunk buckets, thread i of a block taking buckets 4i .. 4i+3 of its
// chunk.  The first writes the sizes into caps and each chunk's sum; the
// second adds the sums of the chunks before its own to a block scan of its
// sizes.  (One block took 41 us at 65536 buckets, bound by what one CU's
// loads and stores can move.)
__global__ __launch_bounds__(kScanThreads) void capacity_sizes_kernel(const uint32_t* __restrict__ hist, uint64_t S,
                                                                      uint64_t n, uint32_t B, double scale,
                                                                      uint32_t* __restrict__ caps,
                                                                      ScanPart* __restrict__ psum,
                                                                      PartHeader* __restrict__ ph,
                                                                      uint64_t cap_slots) {
  __shared__ uint64_t sh[kScanWaves + 1];
  const uint32_t j = blockIdx.x * kScanChunk + 4 * threadIdx.x;
  const double ideal = (double)n / (double)B, per = (double)n / (double)S;
  uint32_t c[4] = {0u, 0u, 0u, 0u};
  if (j + 4 <= B) {
    const uint4 x = *reinterpret_cast<const uint4*>(hist + j);
    c[0] = region_slots(x.x, per, ideal, scale);
    c[1] = region_slots(x.y, per, ideal, scale);
    c[2] = region_slots(x.z, per, ideal, scale);
    c[3] = region_slots(x.w, per, ideal, scale);
    *reinterpret_cast<uint4*>(caps + j) = make_uint4(c[0], c[1], c[2], c[3]);
  } else {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q)
      if (j + q < B) caps[j + q] = c[q] = region_slots(hist[j + q], per, ideal, scale);
  }
  uint64_t tot;
  block_exclusive_scan<uint64_t, kScanThreads>((uint64_t)c[0] + c[1] + c[2] + c[3], sh, &tot);
  if (threadIdx.x == 0) {
    psum[blockIdx.x].c = tot;
    if (blockIdx.x == 0) init_part_header(ph, n, cap_slots, B);
  }
}

__global__ __launch_bounds__(kScanThreads) void capacity_starts_kernel(uint32_t B, uint32_t* __restrict__ caps,
                                                                       uint32_t* __restrict__ rstart,
                                                                       uint32_t* __restrict__ counts, uint32_t cstride,
                                                                       const ScanPart* __restrict__ psum,
                                                                       uint64_t cap_slots) {
  __shared__ uint64_t sh[kScanWaves + 1];
  const uint32_t j = blockIdx.x * kScanChunk + 4 * threadIdx.x;
  uint64_t before = 0;  // the chunks ahead of this one
  for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads) before += psum[i].c;
  uint64_t tot;
  block_exclusive_scan<uint64_t, kScanThreads>(before, sh, &tot);
  before = tot;
  uint32_t c[4] = {0u, 0u, 0u, 0u};
  if (j + 4 <= B) {
    const uint4 x = *reinterpret_cast<const uint4*>(caps + j);
    c[0] = x.x; c[1] = x.y; c[2] = x.z; c[3] = x.w;
  } else {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) c[q] = j + q < B ? caps[j + q] : 0u;
  }
  uint64_t r = before + block_exclusive_scan<uint64_t, kScanThreads>((uint64_t)c[0] + c[1] + c[2] + c[3], sh, &tot);
  uint32_t cp[4], rp[4];
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    const bool fits = r + c[q] <= cap_slots;
    cp[q] = fits ? c[q] : 0u;
    rp[q] = fits ? (uint32_t)r : 0u;
    r += c[q];
  }
  if (j + 4 <= B) {
    *reinterpret_cast<uint4*>(caps + j) = make_uint4(cp[0], cp[1], cp[2], cp[3]);
    *reinterpret_cast<uint4*>(rstart + j) = make_uint4(rp[0], rp[1], rp[2], rp[3]);
    if (cstride == 1) {
      *reinterpret_cast<uint4*>(counts + j) = make_uint4(0, 0, 0, 0);
    } else {
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) counts[(uint64_t)(j + q) * cstride] = 0;
    }
  } else {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      if (j + q < B) {
        caps[j + q] = cp[q];
        rstart[j + q] = rp[q];
        counts[(uint64_t)(j + q) * cstride] = 0;
      }
    }
  }
}

hipError_t launch_capacities(const uint32_t* hist, uint64_t S, uint64_t n, uint32_t B, uint32_t region_pct,
                             uint8_t* part, const PartLayout& lay, hipStream_t st) {
  if (B >= kScanMultiMin) {
    const uint32_t g = (B + kScanChunk - 1) / kScanChunk;
    ScanPart* ps = reinterpret_cast<ScanPart*>(part + lay.psum);
    capacity_sizes_kernel<<<g, kScanThreads, 0, st>>>(hist, S, n, B, region_pct / 100.0,
                                                      reinterpret_cast<uint32_t*>(part + lay.caps), ps,
                                                      reinterpret_cast<PartHeader*>(part + lay.header),
                                                      lay.cap_slots);
    capacity_starts_kernel<<<g, kScanThreads, 0, st>>>(B, reinterpret_cast<uint32_t*>(part + lay.caps),
                                                       reinterpret_cast<uint32_t*>(part + lay.rstart),
                                                       reinterpret_cast<uint32_t*>(part + lay.pcounts), lay.cstride,
                                                       ps, lay.cap_slots);
    return hipGetLastError();
  }
  capacity_kernel<<<1, kScanThreads, 0, st>>>(hist, S, n, B, region_pct / 100.0,
                                              reinterpret_cast<uint32_t*>(part + lay.caps),
                                              reinterpret_cast<uint32_t*>(part + lay.rstart),
                                              reinterpret_cast<uint32_t*>(part + lay.pcounts), lay.cstride,
                                              reinterpret_cast<PartHeader*>(part + lay.header), lay.cap_slots);
  return hipGetLastError();
}

}  // namespace elsar
