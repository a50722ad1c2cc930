// Partition pass (gfx950): predict-and-place of every record (Section 3.3 and
// Algorithm 1's reader loop), the partition sizes S_p and the exclusive output
// offsets of Section 3.5, and the spill fix-up.
//
// Each block stages a tile of records in LDS with coalesced 16-byte loads,
// computes every record's base-95 code and RMI bucket, reserves a slot in the
// bucket's region with one atomic, and writes the record plus its input index
// as one whole 128-byte slot (eight lanes, one 16-byte store each).  A
// bucket that outgrows its region continues in a shared spill area; the
// spill entry remembers (bucket, rank within the bucket's overflow) so the
// fix-up can group the spill without sorting it.
#include <algorithm>
#include <type_traits>

#include "mlp_device.h"

namespace elsar {

constexpr int kPartThreads = 256;
constexpr int kPartTile = 256;  // records per tile (one per thread for the model step)

// Chunk c (16 bytes) of the slot of tile record k: the index, the record
// dwords, then zeros.
__device__ __forceinline__ u32x4 slot_chunk(const uint32_t* tile, uint32_t RW, uint32_t k, uint32_t c, uint32_t idx) {
  u32x4 v;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    uint32_t d = 4 * c + i;  // slot dword
    v[i] = d == 0 ? idx : (d <= RW ? tile[k * RW + d - 1] : 0u);
  }
  return v;
}

// Tile t of records held in registers as RV <= 8 named 16-byte vectors per
// thread plus one dword of tail (named members, not an array, so the compiler
// never demotes them to scratch memory).
struct TileRegs {
  u32x4 v0, v1, v2, v3, v4, v5, v6, v7;
  uint32_t tail;
};
#define ELSAR_FOR8(M) M(0) M(1) M(2) M(3) M(4) M(5) M(6) M(7)

template <uint32_t RV>
__device__ __forceinline__ void load_tile_regs(const uint32_t* __restrict__ rec_dw, uint64_t t, uint32_t cnt,
                                               uint32_t RW, TileRegs& R) {
  static_assert(RV <= 8, "at most 8 vectors per thread");
  const uint32_t ndw = cnt * RW, nvec = ndw >> 2;  // nvec >= 1
  const uint32_t* base = rec_dw + t * kPartTile * RW;
  const u32x4* src4 = reinterpret_cast<const u32x4*>(base);  // 16-byte aligned
  // unconditional loads (index clamped to the last vector): no branches
#define ELSAR_LD(I)                                              \
  if constexpr (I < RV) {                                        \
    uint32_t v = threadIdx.x + (I) * kPartThreads;               \
    R.v##I = __builtin_nontemporal_load(src4 + (v < nvec ? v : nvec - 1)); \
  }
  ELSAR_FOR8(ELSAR_LD)
#undef ELSAR_LD
  uint32_t d = (nvec << 2) + threadIdx.x;
  R.tail = d < ndw ? base[d] : 0u;
}

template <uint32_t RV>
__device__ __forceinline__ void store_tile_regs(uint32_t cnt, uint32_t RW, const TileRegs& R, uint32_t* b) {
  const uint32_t ndw = cnt * RW, nvec = ndw >> 2;
  u32x4* b4 = reinterpret_cast<u32x4*>(b);
  // a clamped index rewrites the last vector with the value its owner writes too
#define ELSAR_ST(I)                                              \
  if constexpr (I < RV) {                                        \
    uint32_t v = threadIdx.x + (I) * kPartThreads;               \
    b4[v < nvec ? v : nvec - 1] = R.v##I;                        \
  }
  ELSAR_FOR8(ELSAR_ST)
#undef ELSAR_ST
  uint32_t d = (nvec << 2) + threadIdx.x;
  if (d < ndw) b[d] = R.tail;
}

// The records are read with nontemporal loads, and the slots written with
// nontemporal stores under the equi-depth and MLP roots: they stream through
// once, and marking them so keeps the routing tables (boundaries, cell
// tables; up to a few MB) resident in L2, where every record's bucket search
// reads them (the spline root's partition went from 8.6 to 8.0 ms at 100M
// skewed records, the linear root's from 5.7 to 5.4 ms at 100M uniform
// ones).  The linear root's tables are small (4096 leaves, 128 KB), and for
// one large job its slots go out as plain stores: 5.45 -> 5.35 ms at 100M
// uniform records (plain loads as well: 5.7-6.2 ms; plain stores under the
// spline root: 6.30 -> 6.45 ms on the skewed law; in the batch's windows:
// 221.6 -> 225.6 ms, so they keep nontemporal stores, as does the host
// tier's filtered pass).
//
// Software pipeline per block over its tiles t = bid, bid + nblk, ... (bid
// and nblk: the block's index and the number of blocks working for the job):
// the loads of tile t+1 are in flight while the atomics of tile t reserve
// slots and the slots of tile t-1 are written, so neither the load latency nor
// the atomic latency stalls the block.  Two LDS tile buffers alternate.
//
// ROOT (kind_used of the header): 0 the linear RMI root; 1 the monotone MLP,
// whose output cell floor(L y) names, through the fit's cell table, a bracket
// of leaves searched among the routing boundaries; 2 the linear spline over
// equi-depth leaves, whose leaf is found among the routing boundaries in the
// bracket of the code's cell (cell_exact_leaf).  A fit
// that may choose among roots launches a kernel per root; each returns at
// once unless the header names its own.
//
// FILTER (host tier): the records are one chunk of a larger input whose first
// record has index f.idx_base; only buckets f.lo .. f.hi-1 are placed (bucket
// b at local bucket b - f.lo), the others are skipped.
template <int RW_T, int ROOT, bool FILTER, bool PLAIN_SLOTS = false>
__device__ __forceinline__ void partition_body(
    const ModelHeader* __restrict__ hdr, const Leaf* __restrict__ leaves, const MlpBlock* __restrict__ mlp,
    const uint64_t* __restrict__ bound, const uint32_t* __restrict__ ccells, const uint32_t* __restrict__ cells,
    const uint8_t* __restrict__ recs, uint64_t n, uint32_t rw_rt, uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps,
    const uint32_t* __restrict__ rstart, PartHeader* __restrict__ ph, uint2* __restrict__ spill_meta,
    uint4* __restrict__ slots, uint64_t cap_slots, PassFilter f, uint32_t vk, uint32_t cstride, uint32_t bid,
    uint32_t nblk) {
  const uint32_t RW = RW_T ? (uint32_t)RW_T : rw_rt;  // record dwords
  const uint32_t SC = slot_bytes_for(RW * 4) / 16;     // 16-byte chunks per slot
  constexpr uint32_t RV = RW_T ? (kPartTile * RW_T / 4 + kPartThreads - 1) / kPartThreads : 8;
  extern __shared__ uint4 lds4[];                      // 2 tiles of kPartTile * RW dwords
  __shared__ uint32_t dst[2][kPartTile];
  constexpr bool MLP = ROOT == 1;
  constexpr bool HOIST = ROOT == 0;
  if (hdr->kind_used != (uint32_t)ROOT) return;
  const uint32_t tile_dw = kPartTile * RW;
  const float a0 = hdr->a0, a1 = hdr->a1;
  const uint32_t L = ROOT ? hdr->mlp_L : hdr->L;
  // equi-depth leaves, one per bucket: floor(B * the spline's CDF) is the leaf
  const bool leaf_is_bucket = ROOT != 0 && L == hdr->B;
  const uint32_t csh = ROOT == 2 ? hdr->cell_shift : 0u;  // the code-cell table of the spline root
  const uint32_t cnc = ROOT == 2 ? code_cells_for(L) : 1u;
  const uint64_t ce0 = ROOT == 2 && L >= 2 ? bound[1] : 0ull;
  __shared__ typename std::conditional<MLP, MlpHead, uint32_t>::type mh_;
  MlpFrags w2;
  if constexpr (MLP) {
    for (uint32_t i = threadIdx.x; i < sizeof(MlpHead) / 4; i += kPartThreads)
      reinterpret_cast<uint32_t*>(&mh_)[i] = reinterpret_cast<const uint32_t*>(&mlp->h)[i];
    mlp_load_frags(mlp, w2);
  }
  const uint64_t ntiles = (n + kPartTile - 1) / kPartTile;
  const uint32_t* rec_dw = reinterpret_cast<const uint32_t*>(recs);
  auto tile_count = [&](uint64_t t) {
    uint64_t r0 = t * kPartTile;
    return (uint32_t)(n - r0 < (uint64_t)kPartTile ? n - r0 : (uint64_t)kPartTile);
  };
  auto buf = [&](uint32_t i) { return reinterpret_cast<uint32_t*>(lds4) + i * tile_dw; };
  // SC consecutive lanes write one slot as whole 16-byte chunks (whole lines)
  auto write_tile = [&](uint64_t t, const uint32_t* b, const uint32_t* dslot) {
    const uint32_t total = tile_count(t) * SC;
    const uint32_t r0 = (uint32_t)(FILTER ? f.idx_base + t * kPartTile : t * kPartTile);
    for (uint32_t q = threadIdx.x; q < total; q += kPartThreads) {
      uint32_t k = q / SC, c = q - k * SC;
      if (FILTER && dslot[k] == kNoSlot) continue;
      u32x4* dst = reinterpret_cast<u32x4*>(slots) + (uint64_t)dslot[k] * SC + c;
      if (PLAIN_SLOTS) *dst = slot_chunk(b, RW, k, c, r0 + k);
      else __builtin_nontemporal_store(slot_chunk(b, RW, k, c, r0 + k), dst);
    }
  };

  uint64_t t = bid;
  if (t >= ntiles) return;
  // tile t is copied through registers: RV 16-byte vectors per thread plus a dword tail
  {
    TileRegs R;
    load_tile_regs<RV>(rec_dw, t, tile_count(t), RW, R);
    store_tile_regs<RV>(tile_count(t), RW, R, buf(0));
  }
  __syncthreads();
  uint32_t cur = 0;
  bool have_prev = false;
  uint64_t tprev = 0;
  for (;;) {
    const uint64_t tn = t + nblk;
    const bool have_next = tn < ntiles;
    // 1. loads of the next tile (the last iteration reloads its own tile
    //    instead: no branch around the loads), and 2. the bucket of each
    //    record of tile t
    const uint64_t tl = have_next ? tn : t;
    const uint32_t cnt = tile_count(t);
    uint32_t b = 0, s = 0;
    TileRegs R;
    if constexpr (ROOT == 0) {
      // Under the linear root the leaf line's load goes out before the next
      // tile's loads and stays ahead of them (the scheduling barriers): loads
      // complete in issue order, so the wait for the leaf does not include
      // the wait for the tile (5.17 -> 5.14 ms at 100M uniform records).
      // Lanes past the tile's end route stale bytes to a leaf in range and
      // discard the result.
      const uint32_t* r = buf(cur) + threadIdx.x * RW;
      uint32_t r0 = r[0], r1 = r[1], r2 = vk ? r[2] : 0u;
      virtual_key(r0, r1, r2, vk);
      const uint64_t e = key_code(r0, r1);
      const Leaf lf = load_leaf(leaves, rmi_leaf(a0, a1, L, e));
      __builtin_amdgcn_sched_barrier(0);
      load_tile_regs<RV>(rec_dw, tl, tile_count(tl), RW, R);
      __builtin_amdgcn_sched_barrier(0);
      b = leaf_bucket(lf, e);
    } else {
      // the spline and MLP roots' searches overlap the next tile's loads
      // (issued after the searches, the skewed law's whole sort took 13.4 ms
      // instead of 12.1)
      load_tile_regs<RV>(rec_dw, tl, tile_count(tl), RW, R);
      uint64_t e = 0;
      Leaf lf{};
      if constexpr (MLP) {
        // every lane takes part in the matrix products; lanes past the tile's
        // end read stale tile bytes and discard the result
        const uint32_t* r = buf(cur) + threadIdx.x * RW;
        uint32_t r0 = r[0], r1 = r[1], r2 = vk ? r[2] : 0u;
        virtual_key(r0, r1, r2, vk);
        e = key_code(r0, r1);
        const float y = mlp_y64(e, mh_, w2);
        if (threadIdx.x < cnt) {
          const uint32_t j = mlp_bracket_leaf(bound, cells, L, e, y);
          if (leaf_is_bucket) b = j;
          else lf = load_leaf(leaves, j);
        }
      } else if (threadIdx.x < cnt) {
        const uint32_t* r = buf(cur) + threadIdx.x * RW;
        uint32_t r0 = r[0], r1 = r[1], r2 = vk ? r[2] : 0u;
        virtual_key(r0, r1, r2, vk);
        e = key_code(r0, r1);
        const uint32_t j = cell_exact_leaf(ccells, csh, cnc, ce0, bound, e);
        if (leaf_is_bucket) b = j;
        else lf = load_leaf(leaves, j);
      }
      if (!leaf_is_bucket && threadIdx.x < cnt) b = leaf_bucket(lf, e);
    }
    bool keep = threadIdx.x < cnt;
    if (FILTER) {
      keep = keep && b >= f.lo && b < f.hi;
      b -= f.lo;
    }
    // Under the linear root the region's size and start travel with the
    // atomic: loaded after it returned, they were two more dependent trips to
    // L2 (5.34 -> 5.17 ms at 100M uniform records).  Under the spline and MLP
    // roots the same order measured slower (6.18 -> 6.5-6.7 ms on the skewed
    // law), so they keep the loads after the atomic.
    uint32_t cap = 0, rs = 0;
    if (keep) {
      if (HOIST) {
        cap = caps[b];
        rs = rstart[b];
      }
      s = atomicAdd(&counts[(uint64_t)b * cstride], 1u);
    }
    // 3. the previous tile's slots, while the atomics are in flight
    if (have_prev) write_tile(tprev, buf(cur ^ 1), dst[cur ^ 1]);
    // 4. this tile's slots.  Overflowing records take spill positions from one
    //    shared counter; a wave reserves all of its own with a single atomic
    //    (skewed inputs overflow in bursts, and same-address atomics serialise).
    uint32_t slot = kNoSlot, over = 0;
    bool spill = false;
    if (keep) {
      if (!HOIST) cap = caps[b];
      if (s < cap) slot = (HOIST ? rs : rstart[b]) + s;
      else { spill = true; over = s - cap; }
    }
    const uint64_t spill_mask = __ballot(spill);
    if (spill_mask) {
      const uint32_t leader = (uint32_t)__ffsll((long long)spill_mask) - 1u;
      uint32_t q0 = 0;
      if (lane_id() == leader) q0 = atomicAdd(&ph->spill_count, (uint32_t)__popcll(spill_mask));
      q0 = __shfl(q0, (int)leader);
      // FILTER: exact regions leave no room, so an overflow is only counted (an
      // error for the caller) and never placed
      if (!FILTER && spill) {
        const uint32_t q = q0 + (uint32_t)__popcll(spill_mask & lanemask_lt());
        spill_meta[q] = make_uint2(b, over);
        slot = (uint32_t)cap_slots + q;
      }
    }
    if (threadIdx.x < cnt) dst[cur][threadIdx.x] = slot;
    __syncthreads();
    // 5. the next tile into the buffer the previous tile has left (on the last
    //    iteration a copy of tile t lands there unused; again no branch)
    store_tile_regs<RV>(tile_count(tl), RW, R, buf(cur ^ 1));
    __syncthreads();
    have_prev = true;
    tprev = t;
    if (!have_next) break;
    t = tn;
    cur ^= 1;
  }
  write_tile(tprev, buf(cur), dst[cur]);
}

template <int RW_T, int ROOT, bool FILTER>
__global__ __launch_bounds__(kPartThreads) void partition_kernel(
    const ModelHeader* __restrict__ hdr, const Leaf* __restrict__ leaves, const MlpBlock* __restrict__ mlp,
    const uint64_t* __restrict__ bound, const uint32_t* __restrict__ ccells, const uint32_t* __restrict__ cells,
    const uint8_t* __restrict__ recs, uint64_t n, uint32_t rw_rt, uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps,
    const uint32_t* __restrict__ rstart, PartHeader* __restrict__ ph, uint2* __restrict__ spill_meta,
    uint4* __restrict__ slots, uint64_t cap_slots, PassFilter f, uint32_t vk, uint32_t cstride) {
  // one job under the linear root: plain slot stores (see above)
  partition_body<RW_T, ROOT, FILTER, ROOT == 0 && !FILTER>(hdr, leaves, mlp, bound, ccells, cells, recs, n, rw_rt,
                                                           counts, caps, rstart, ph, spill_meta, slots, cap_slots, f,
                                                           vk, cstride, blockIdx.x, gridDim.x);
}

// A window of a batch: G blocks per job.
template <int RW_T, int ROOT>
__global__ __launch_bounds__(kPartThreads) void partition_win_kernel(const WinJob* __restrict__ jobs, uint32_t G,
                                                                     uint32_t rw_rt) {
  const WinJob& J = jobs[blockIdx.x / G];
  uint8_t* part = J.part;
  partition_body<RW_T, ROOT, false>(
      J.hdr, ROOT ? J.eq_leaves : J.leaves, J.mlp, J.bound, J.ccells, J.cells, J.recs, J.n, rw_rt,
      reinterpret_cast<uint32_t*>(part + J.lay.pcounts), reinterpret_cast<const uint32_t*>(part + J.lay.caps),
      reinterpret_cast<const uint32_t*>(part + J.lay.rstart), reinterpret_cast<PartHeader*>(part + J.lay.header),
      reinterpret_cast<uint2*>(part + J.lay.spill_meta), reinterpret_cast<uint4*>(part + J.lay.slots),
      J.lay.cap_slots, PassFilter{0, 0, 0}, 0u, J.lay.cstride, blockIdx.x % G, G);
}

// Blocks of the partition of n records: at least four tiles per block below
// 8192 tiles, so that the pipeline has tiles to overlap (small jobs of a
// batch run beside others), at most 2048 blocks.
uint32_t partition_grid(uint64_t n) {
  const uint64_t ntiles = (n + kPartTile - 1) / kPartTile;
  return ntiles < 8192 ? (uint32_t)((ntiles + 3) / 4) : 2048u;
}

template <int ROOT, bool FILTER>
static void launch_partition_root(uint32_t grid, size_t lds, hipStream_t st, uint32_t RW, const ModelHeader* hdr,
                                  const Leaf* leaves, const MlpBlock* mlp, const uint64_t* bound,
                                  const uint32_t* ccells, const uint32_t* cells, const uint8_t* recs, uint64_t n,
                                  uint32_t* counts,
                                  const uint32_t* caps, const uint32_t* rstart, PartHeader* ph, uint2* meta,
                                  uint4* slots, uint64_t cap_slots, PassFilter f, uint32_t vk, uint32_t cstride) {
  if (RW == 25)
    partition_kernel<25, ROOT, FILTER><<<grid, kPartThreads, lds, st>>>(hdr, leaves, mlp, bound, ccells, cells, recs, n, RW,
                                                                        counts, caps, rstart, ph, meta, slots,
                                                                        cap_slots, f, vk, cstride);
  else
    partition_kernel<0, ROOT, FILTER><<<grid, kPartThreads, lds, st>>>(hdr, leaves, mlp, bound, ccells, cells, recs, n, RW,
                                                                       counts, caps, rstart, ph, meta, slots,
                                                                       cap_slots, f, vk, cstride);
}

hipError_t launch_partition(const ModelHeader* hdr, const Leaf* leaves, const MlpState* ms, const uint8_t* recs,
                            uint64_t n, uint32_t rec_bytes, uint32_t vk, uint8_t* part,
                            const PartLayout& lay, hipStream_t st, const PassFilter* filter) {
  if (n == 0) return hipSuccess;
  const uint32_t RW = rec_bytes / 4;
  const size_t lds = 2 * (size_t)kPartTile * RW * 4;
  const uint32_t grid = partition_grid(n);
  auto* counts = reinterpret_cast<uint32_t*>(part + lay.pcounts);  // the partition's slot counters
  const uint32_t cstride = lay.cstride;
  auto* caps = reinterpret_cast<const uint32_t*>(part + lay.caps);
  auto* rstart = reinterpret_cast<const uint32_t*>(part + lay.rstart);
  auto* ph = reinterpret_cast<PartHeader*>(part + lay.header);
  auto* meta = reinterpret_cast<uint2*>(part + lay.spill_meta);
  auto* slots = reinterpret_cast<uint4*>(part + lay.slots);
  const PassFilter f = filter ? *filter : PassFilter{0, 0, 0};
  if (filter) {
    launch_partition_root<0, true>(grid, lds, st, RW, hdr, leaves, nullptr, nullptr, nullptr, nullptr, recs, n,
                                   counts, caps, rstart, ph, meta, slots, lay.cap_slots, f, vk, cstride);
    if (ms) {
      launch_partition_root<1, true>(grid, lds, st, RW, hdr, ms->leaves, ms->M, ms->bound, nullptr, ms->cells, recs,
                                     n, counts, caps, rstart, ph, meta, slots, lay.cap_slots, f, vk, cstride);
      launch_partition_root<2, true>(grid, lds, st, RW, hdr, ms->leaves, nullptr, ms->bound, ms->ccells, nullptr, recs,
                                     n, counts, caps, rstart, ph, meta, slots, lay.cap_slots, f, vk, cstride);
    }
  } else {
    launch_partition_root<0, false>(grid, lds, st, RW, hdr, leaves, nullptr, nullptr, nullptr, nullptr, recs, n,
                                    counts, caps, rstart, ph, meta, slots, lay.cap_slots, f, vk, cstride);
    if (ms) {
      launch_partition_root<1, false>(grid, lds, st, RW, hdr, ms->leaves, ms->M, ms->bound, nullptr, ms->cells, recs,
                                      n, counts, caps, rstart, ph, meta, slots, lay.cap_slots, f, vk, cstride);
      launch_partition_root<2, false>(grid, lds, st, RW, hdr, ms->leaves, nullptr, ms->bound, ms->ccells, nullptr,
                                      recs, n, counts, caps, rstart, ph, meta, slots, lay.cap_slots, f, vk, cstride);
    }
  }
  return hipGetLastError();
}

template <int RW_T>
static void launch_partition_win_rw(const WinJob* jobs, uint32_t njobs, uint32_t G, uint32_t RW, bool equi_depth,
                                    hipStream_t st) {
  const size_t lds = 2 * (size_t)kPartTile * RW * 4;
  partition_win_kernel<RW_T, 0><<<njobs * G, kPartThreads, lds, st>>>(jobs, G, RW);
  if (equi_depth) {
    partition_win_kernel<RW_T, 1><<<njobs * G, kPartThreads, lds, st>>>(jobs, G, RW);
    partition_win_kernel<RW_T, 2><<<njobs * G, kPartThreads, lds, st>>>(jobs, G, RW);
  }
}

hipError_t launch_partition_win(const WinJob* jobs, uint32_t njobs, uint32_t G, uint32_t rec_bytes, bool equi_depth,
                                hipStream_t st) {
  if (njobs == 0 || G == 0) return hipSuccess;
  const uint32_t RW = rec_bytes / 4;
  if (RW == 25)
    launch_partition_win_rw<25>(jobs, njobs, G, RW, equi_depth, st);
  else
    launch_partition_win_rw<0>(jobs, njobs, G, RW, equi_depth, st);
  return hipGetLastError();
}

// ------------------------------------------------------------- host tier --
// Bucket counts of one chunk of records (no placement).  A wave takes 64
// consecutive records; lanes past the end evaluate a clamped copy and drop it.
template <int ROOT>
__global__ __launch_bounds__(256) void count_kernel(const ModelHeader* __restrict__ hdr,
                                                    const Leaf* __restrict__ leaves, const MlpBlock* __restrict__ mlp,
                                                    const uint64_t* __restrict__ bound,
                                                    const uint32_t* __restrict__ ccells,
                                                    const uint32_t* __restrict__ cells, const uint32_t* __restrict__ rec,
                                                    uint64_t n, uint32_t RW, uint32_t* __restrict__ counts,
                                                    uint32_t vk) {
  constexpr bool MLP = ROOT == 1;
  if (hdr->kind_used != (uint32_t)ROOT) return;
  __shared__ typename std::conditional<MLP, MlpHead, uint32_t>::type mh_;
  MlpFrags w2;
  if constexpr (MLP) {
    for (uint32_t i = threadIdx.x; i < sizeof(MlpHead) / 4; i += blockDim.x)
      reinterpret_cast<uint32_t*>(&mh_)[i] = reinterpret_cast<const uint32_t*>(&mlp->h)[i];
    mlp_load_frags(mlp, w2);
    __syncthreads();
  }
  const float a0 = hdr->a0, a1 = hdr->a1;
  const uint32_t L = ROOT ? hdr->mlp_L : hdr->L;
  const uint32_t csh = ROOT == 2 ? hdr->cell_shift : 0u;
  const uint32_t cnc = ROOT == 2 ? code_cells_for(L) : 1u;
  const uint64_t ce0 = ROOT == 2 && L >= 2 ? bound[1] : 0ull;
  const bool leaf_is_bucket = ROOT != 0 && L == hdr->B;
  const uint64_t wave0 = ((uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u));
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t base = wave0; base < n; base += stride) {  // uniform per wave
    const uint64_t i = base + lane_id();
    const uint32_t* r = rec + (i < n ? i : n - 1) * RW;
    uint32_t r0 = r[0], r1 = r[1], r2 = vk ? r[2] : 0u;
    virtual_key(r0, r1, r2, vk);
    const uint64_t e = key_code(r0, r1);
    uint32_t b;
    if constexpr (MLP) {
      const float y = mlp_y64(e, mh_, w2);
      const uint32_t j = mlp_bracket_leaf(bound, cells, L, e, y);
      b = leaf_is_bucket ? j : leaf_bucket(load_leaf(leaves, j), e);
    } else {
      const uint32_t j = ROOT == 2 ? cell_exact_leaf(ccells, csh, cnc, ce0, bound, e) : rmi_leaf(a0, a1, L, e);
      b = leaf_is_bucket ? j : leaf_bucket(load_leaf(leaves, j), e);
    }
    if (i < n) atomicAdd(&counts[b], 1u);
  }
}

hipError_t launch_count(const ModelHeader* hdr, const Leaf* leaves, const MlpState* ms, const uint8_t* recs,
                        uint64_t n, uint32_t rec_bytes, uint32_t* counts, hipStream_t st, uint32_t vk) {
  if (n == 0) return hipSuccess;
  const uint32_t RW = rec_bytes / 4;
  const uint64_t waves = (n + 63) / 64;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((waves + 3) / 4, 4096);
  const uint32_t* rec = reinterpret_cast<const uint32_t*>(recs);
  count_kernel<0><<<grid, 256, 0, st>>>(hdr, leaves, nullptr, nullptr, nullptr, nullptr, rec, n, RW, counts, vk);
  if (ms) {
    count_kernel<1><<<grid, 256, 0, st>>>(hdr, ms->leaves, ms->M, ms->bound, nullptr, ms->cells, rec, n, RW, counts, vk);
    count_kernel<2><<<grid, 256, 0, st>>>(hdr, ms->leaves, nullptr, ms->bound, ms->ccells, nullptr, rec, n, RW,
                                          counts, vk);
  }
  return hipGetLastError();
}

// flag[0] = 1 if the first K bytes of any of n records differ from ref (the
// host tier's check of a bucket that it copies through without sorting).
__global__ __launch_bounds__(256) void keys_differ_kernel(const uint8_t* __restrict__ recs, uint64_t n, uint32_t R,
                                                          uint32_t K, const uint8_t* __restrict__ ref,
                                                          uint32_t* __restrict__ flag) {
  bool diff = false;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint8_t* r = recs + i * R;
    for (uint32_t b = 0; b < K; ++b) diff |= r[b] != ref[b];
  }
  if (__ballot(diff) && lane_id() == 0) flag[0] = 1u;
}

hipError_t launch_keys_differ(const uint8_t* recs, uint64_t n, uint32_t rec_bytes, uint32_t key_bytes,
                              const uint8_t* ref, uint32_t* flag, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = (uint32_t)std::min<uint64_t>((n + 255) / 256, 4096);
  keys_differ_kernel<<<grid, 256, 0, st>>>(recs, n, rec_bytes, key_bytes, ref, flag);
  return hipGetLastError();
}

// One pass of the host tier places buckets lo .. hi-1 in exact regions:
// caps[j] = counts_all[lo + j], rstart = their exclusive sum, counts zeroed,
// header set for total records and hi - lo buckets.  One block.
constexpr uint32_t kExThreads = 1024;
constexpr uint32_t kExPer = 8;

__global__ __launch_bounds__(kExThreads) void exact_regions_kernel(const uint32_t* __restrict__ counts_all,
                                                                   uint32_t lo, uint32_t nb, uint64_t total,
                                                                   uint32_t* __restrict__ caps,
                                                                   uint32_t* __restrict__ rstart,
                                                                   uint32_t* __restrict__ counts, uint32_t cstride,
                                                                   PartHeader* __restrict__ ph) {
  __shared__ uint64_t sh[kExThreads / 64 + 1];
  uint64_t carry = 0;
  for (uint32_t base = 0; base < nb; base += kExThreads * kExPer) {
    uint32_t c[kExPer];
    uint64_t sum = 0;
#pragma unroll
    for (uint32_t i = 0; i < kExPer; ++i) {
      const uint32_t j = base + threadIdx.x * kExPer + i;
      c[i] = j < nb ? counts_all[lo + j] : 0u;
      sum += c[i];
    }
    uint64_t tot;
    uint64_t run = block_exclusive_scan<uint64_t, kExThreads>(sum, sh, &tot) + carry;
#pragma unroll
    for (uint32_t i = 0; i < kExPer; ++i) {
      const uint32_t j = base + threadIdx.x * kExPer + i;
      if (j < nb) {
        caps[j] = c[i];
        rstart[j] = (uint32_t)run;
        counts[(uint64_t)j * cstride] = 0;
      }
      run += c[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    ph->n = total;
    ph->cap_slots = total;
    ph->B = nb;
    ph->spill_count = 0;
    ph->n_mid = 0;
    ph->n_mid_hi = 0;
    ph->n_big = 0;
    ph->n_big2 = 0;
    ph->max_count = 0;
    ph->mid_records = 0;
    ph->big_records = 0;
  }
}

hipError_t launch_exact_regions(const uint32_t* counts_all, uint32_t lo, uint32_t nb, uint64_t total, uint8_t* part,
                                const PartLayout& lay, hipStream_t st) {
  exact_regions_kernel<<<1, kExThreads, 0, st>>>(counts_all, lo, nb, total,
                                                 reinterpret_cast<uint32_t*>(part + lay.caps),
                                                 reinterpret_cast<uint32_t*>(part + lay.rstart),
                                                 reinterpret_cast<uint32_t*>(part + lay.pcounts), lay.cstride,
                                                 reinterpret_cast<PartHeader*>(part + lay.header));
  return hipGetLastError();
}

// offsets[j] = sum_{k<j} counts[k] (u64), offsets[B] = n; spill_off[j] = sum_{k<j}
// max(counts[k] - caps[k], 0); buckets above the small LDS cap go to lists.
// One block.  Wave w owns a contiguous segment of WS buckets (WS a multiple of
// 1024) and walks it 256 buckets a step, lane l taking buckets 4l .. 4l+3 of
// the step, so that every load and store of the wave covers whole lines; the
// loads of four steps are issued before any is used.  Pass 1 sums the wave's
// counts and overflows; the waves' sums are scanned in order; pass 2 scans
// each step across the wave and writes the offsets.
constexpr uint32_t kScanThreads = 1024;
constexpr uint32_t kScanWaves = kScanThreads / 64;
constexpr uint32_t kScanSteps = 8;  // steps of 256 buckets whose loads are in flight together

// counts: the partition's slot counters, cstride apart; with cstride > 1 the
// dense counts the bucket sorts read go to dense.
__device__ __forceinline__ void scan_counts_body(const uint32_t* __restrict__ counts, uint32_t cstride,
                                                 uint32_t* __restrict__ dense, const uint32_t* __restrict__ caps,
                                                 uint32_t B, uint64_t* __restrict__ offsets,
                                                 uint32_t* __restrict__ spill_off, uint32_t* __restrict__ mid_list,
                                                 uint32_t* __restrict__ big_list, PartHeader* __restrict__ ph) {
  __shared__ uint64_t shc[kScanWaves + 1];
  __shared__ uint32_t shs[kScanWaves];
  __shared__ uint32_t sh_nmid, sh_nmid_hi, sh_nbig;  // list lengths: LDS atomics (one global address would serialise them)
  if (threadIdx.x == 0) {
    sh_nmid = 0;
    sh_nmid_hi = 0;
    sh_nbig = 0;
  }
  __syncthreads();
  const uint32_t WS = ((B + kScanWaves - 1) / kScanWaves + 1023) & ~1023u;
  const uint32_t w = threadIdx.x >> 6, l = lane_id();
  const uint32_t s0 = w * WS, s1 = s0 + WS < B ? s0 + WS : B;  // empty when s0 >= B
  // values of buckets j .. j+3 (zero past the segment), one 16-byte load
  // with no branch around it (a load inside a branch is waited for there,
  // which made the steps' loads one round trip each): past the end of the
  // array it reads its last vector again, and the array's space, rounded up
  // to a multiple of 256 bytes, keeps that vector's tail in bounds
  const uint32_t jlast = (B - 1) & ~3u;
  auto load4 = [&](const uint32_t* src, uint32_t j, uint32_t v[4]) {
    const uint4 x = *reinterpret_cast<const uint4*>(src + (j < B ? j : jlast));
    v[0] = j < s1 ? x.x : 0u;
    v[1] = j + 1 < s1 ? x.y : 0u;
    v[2] = j + 2 < s1 ? x.z : 0u;
    v[3] = j + 3 < s1 ? x.w : 0u;
  };
  // counts of buckets j .. j+3 (zero past the segment), wherever the counters sit
  auto loadc = [&](uint32_t j, uint32_t v[4]) {
    if (cstride == 1) {
      load4(counts, j, v);
    } else {
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t c = counts[(uint64_t)(j + q < B ? j + q : B - 1) * cstride];
        v[q] = j + q < s1 ? c : 0u;
      }
    }
  };
  auto over = [](uint32_t c, uint32_t k) { return c > k ? c - k : 0u; };
  uint64_t sc = 0;
  uint32_t ss = 0, m = 0, mr = 0, br = 0;
  for (uint32_t jb = s0; jb < s1; jb += 256 * kScanSteps) {
    uint32_t c[kScanSteps][4], k[kScanSteps][4];
#pragma unroll
    for (uint32_t u = 0; u < kScanSteps; ++u) {
      loadc(jb + 256 * u + 4 * l, c[u]);
      load4(caps, jb + 256 * u + 4 * l, k[u]);
    }
#pragma unroll
    for (uint32_t u = 0; u < kScanSteps; ++u) {
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        const uint32_t cq = c[u][q];
        sc += cq;
        ss += over(cq, k[u][q]);
        m = cq > m ? cq : m;
        if (cq > kSmallCap) {  // zero past the segment
          const uint32_t j = jb + 256 * u + 4 * l + q;
          if (cq <= kMidLoCap) {  // from the start of the list
            mid_list[atomicAdd(&sh_nmid, 1u)] = j;
            mr += cq;
          } else if (cq <= kMidCap) {  // from its end
            mid_list[B - 1 - atomicAdd(&sh_nmid_hi, 1u)] = j;
            mr += cq;
          } else {
            big_list[atomicAdd(&sh_nbig, 1u)] = j;
            br += cq;
          }
        }
      }
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    sc += shfl_xor_u64(sc, off);
    ss += __shfl_xor(ss, off);
    mr += __shfl_xor(mr, off);
    br += __shfl_xor(br, off);
    const uint32_t mo = __shfl_xor(m, off);
    m = mo > m ? mo : m;
  }
  if (l == 0) {
    shc[w] = sc;
    shs[w] = ss;
    if (mr) atomicAdd(&ph->mid_records, mr);
    if (br) atomicAdd(&ph->big_records, br);
    if (m) atomicMax(&ph->max_count, m);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t rc = 0;
    uint32_t rs = 0;
    for (uint32_t i = 0; i < kScanWaves; ++i) {
      const uint64_t c = shc[i];
      const uint32_t x = shs[i];
      shc[i] = rc;
      shs[i] = rs;
      rc += c;
      rs += x;
    }
    shc[kScanWaves] = rc;
    ph->n_mid = sh_nmid;
    ph->n_mid_hi = sh_nmid_hi;
    ph->n_big = sh_nbig;
  }
  __syncthreads();
  uint64_t rc = shc[w];
  uint32_t rs = shs[w];
  for (uint32_t jb = s0; jb < s1; jb += 256 * kScanSteps) {
    uint32_t c[kScanSteps][4], k[kScanSteps][4];
#pragma unroll
    for (uint32_t u = 0; u < kScanSteps; ++u) {
      loadc(jb + 256 * u + 4 * l, c[u]);
      load4(caps, jb + 256 * u + 4 * l, k[u]);
    }
#pragma unroll
    for (uint32_t u = 0; u < kScanSteps; ++u) {
      const uint32_t j = jb + 256 * u + 4 * l;
      const uint64_t oc = (uint64_t)c[u][0] + c[u][1] + c[u][2] + c[u][3];
      const uint32_t os = over(c[u][0], k[u][0]) + over(c[u][1], k[u][1]) + over(c[u][2], k[u][2]) +
                          over(c[u][3], k[u][3]);
      const uint64_t xc = wave_inclusive_scan<uint64_t>(oc);
      const uint32_t xs = wave_inclusive_scan<uint32_t>(os);
      uint64_t r = rc + xc - oc;
      uint32_t t = rs + xs - os;
      uint32_t so[4];
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) {
        if (j + q < s1) offsets[j + q] = r;
        so[q] = t;
        r += c[u][q];
        t += over(c[u][q], k[u][q]);
      }
      if (j + 4 <= s1) {
        *reinterpret_cast<uint4*>(spill_off + j) = make_uint4(so[0], so[1], so[2], so[3]);
        if (cstride > 1) *reinterpret_cast<uint4*>(dense + j) = make_uint4(c[u][0], c[u][1], c[u][2], c[u][3]);
      } else {
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q)
          if (j + q < s1) {
            spill_off[j + q] = so[q];
            if (cstride > 1) dense[j + q] = c[u][q];
          }
      }
      rc += shfl_u64(xc, 63);  // the step's sums
      rs += __shfl(xs, 63);
    }
  }
  if (threadIdx.x == 0) offsets[B] = shc[kScanWaves];
}

__global__ __launch_bounds__(kScanThreads) void scan_counts_kernel(const uint32_t* __restrict__ counts,
                                                                   uint32_t cstride, uint32_t* __restrict__ dense,
                                                                   const uint32_t* __restrict__ caps, uint32_t B,
                                                                   uint64_t* __restrict__ offsets,
                                                                   uint32_t* __restrict__ spill_off,
                                                                   uint32_t* __restrict__ mid_list,
                                                                   uint32_t* __restrict__ big_list,
                                                                   PartHeader* __restrict__ ph) {
  scan_counts_body(counts, cstride, dense, caps, B, offsets, spill_off, mid_list, big_list, ph);
}

// A window of a batch: one block per job.
__global__ __launch_bounds__(kScanThreads) void scan_counts_win_kernel(const WinJob* __restrict__ jobs) {
  const WinJob& J = jobs[blockIdx.x];
  uint8_t* part = J.part;
  scan_counts_body(reinterpret_cast<const uint32_t*>(part + J.lay.pcounts), J.lay.cstride,
                   reinterpret_cast<uint32_t*>(part + J.lay.counts), reinterpret_cast<const uint32_t*>(part + J.lay.caps),
                   J.B, J.offsets, reinterpret_cast<uint32_t*>(part + J.lay.spill_off),
                   reinterpret_cast<uint32_t*>(part + J.lay.mid_list), reinterpret_cast<uint32_t*>(part + J.lay.big_list),
                   reinterpret_cast<PartHeader*>(part + J.lay.header));
}

hipError_t launch_scan_counts_win(const WinJob* jobs, uint32_t njobs, hipStream_t st) {
  if (njobs == 0) return hipSuccess;
  scan_counts_win_kernel<<<njobs, kScanThreads, 0, st>>>(jobs);
  return hipGetLastError();
}

// Many buckets: the same scan in two launches over chunks of kScanChunk
// buckets, thread i of a block taking buckets 4i .. 4i+3 of its chunk.  The
// first sums each chunk's counts and overflows and lists its large buckets
// (one atomic per list and wave reserves the wave's entries); the second adds
// the sums of the chunks before its own to a block scan of its counts.  (One
// block took 41-51 us at 65536 buckets, bound by what one CU's loads and
// stores can move.)
__device__ __forceinline__ void load_chunk4(const uint32_t* __restrict__ counts, uint32_t cstride,
                                            const uint32_t* __restrict__ caps, uint32_t B, uint32_t j, uint32_t c[4],
                                            uint32_t k[4]) {
  if (j + 4 <= B) {
    const uint4 y = *reinterpret_cast<const uint4*>(caps + j);
    k[0] = y.x; k[1] = y.y; k[2] = y.z; k[3] = y.w;
    if (cstride == 1) {
      const uint4 x = *reinterpret_cast<const uint4*>(counts + j);
      c[0] = x.x; c[1] = x.y; c[2] = x.z; c[3] = x.w;
    } else {
#pragma unroll
      for (uint32_t q = 0; q < 4; ++q) c[q] = counts[(uint64_t)(j + q) * cstride];
    }
  } else {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      c[q] = j + q < B ? counts[(uint64_t)(j + q) * cstride] : 0u;
      k[q] = j + q < B ? caps[j + q] : 0u;
    }
  }
}

__device__ __forceinline__ uint32_t overflow_of(uint32_t c, uint32_t k) { return c > k ? c - k : 0u; }

__global__ __launch_bounds__(kScanThreads) void scan_sums_kernel(const uint32_t* __restrict__ counts, uint32_t cstride,
                                                                 const uint32_t* __restrict__ caps, uint32_t B,
                                                                 uint32_t* __restrict__ mid_list,
                                                                 uint32_t* __restrict__ big_list,
                                                                 PartHeader* __restrict__ ph,
                                                                 ScanPart* __restrict__ psum) {
  __shared__ uint64_t shc[kScanWaves];
  __shared__ uint32_t shs[kScanWaves];
  const uint32_t w = threadIdx.x >> 6, l = lane_id();
  const uint32_t j = blockIdx.x * kScanChunk + 4 * threadIdx.x;
  uint32_t c[4], k[4];
  load_chunk4(counts, cstride, caps, B, j, c, k);
  uint64_t sc = 0;
  uint32_t ss = 0, m = 0, mr = 0, br = 0;
  uint32_t nl = 0;  // this thread's list entries, 10 bits a list: mid, mid from the end, big
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    const uint32_t cq = c[q];  // zero past B
    sc += cq;
    ss += overflow_of(cq, k[q]);
    m = cq > m ? cq : m;
    if (cq > kSmallCap) {
      if (cq <= kMidLoCap) { nl += 1u; mr += cq; }
      else if (cq <= kMidCap) { nl += 1u << 10; mr += cq; }
      else { nl += 1u << 20; br += cq; }
    }
  }
  // at most 256 entries of a list per wave: the 10-bit fields never carry
  const uint32_t incl = wave_inclusive_scan<uint32_t>(nl);
  const uint32_t wtot = __shfl(incl, 63);
  if (wtot) {
    uint32_t b0 = 0, b1 = 0, b2 = 0;
    if (l == 0) {
      if (wtot & 1023u) b0 = atomicAdd(&ph->n_mid, wtot & 1023u);
      if ((wtot >> 10) & 1023u) b1 = atomicAdd(&ph->n_mid_hi, (wtot >> 10) & 1023u);
      if (wtot >> 20) b2 = atomicAdd(&ph->n_big, wtot >> 20);
    }
    const uint32_t ex = incl - nl;
    b0 = __shfl(b0, 0) + (ex & 1023u);
    b1 = __shfl(b1, 0) + ((ex >> 10) & 1023u);
    b2 = __shfl(b2, 0) + (ex >> 20);
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q) {
      const uint32_t cq = c[q];
      if (cq > kSmallCap) {
        if (cq <= kMidLoCap) mid_list[b0++] = j + q;          // from the start of the list
        else if (cq <= kMidCap) mid_list[B - 1 - b1++] = j + q;  // from its end
        else big_list[b2++] = j + q;
      }
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    sc += shfl_xor_u64(sc, off);
    ss += __shfl_xor(ss, off);
    mr += __shfl_xor(mr, off);
    br += __shfl_xor(br, off);
    const uint32_t mo = __shfl_xor(m, off);
    m = mo > m ? mo : m;
  }
  if (l == 0) {
    shc[w] = sc;
    shs[w] = ss;
    if (mr) atomicAdd(&ph->mid_records, mr);
    if (br) atomicAdd(&ph->big_records, br);
    if (m) atomicMax(&ph->max_count, m);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tc = 0;
    uint32_t ts = 0;
    for (uint32_t i = 0; i < kScanWaves; ++i) {
      tc += shc[i];
      ts += shs[i];
    }
    psum[blockIdx.x].c = tc;
    psum[blockIdx.x].s = ts;
  }
}

__global__ __launch_bounds__(kScanThreads) void scan_offsets_kernel(const uint32_t* __restrict__ counts,
                                                                    uint32_t cstride, uint32_t* __restrict__ dense,
                                                                    const uint32_t* __restrict__ caps, uint32_t B,
                                                                    uint64_t* __restrict__ offsets,
                                                                    uint32_t* __restrict__ spill_off,
                                                                    const ScanPart* __restrict__ psum) {
  __shared__ uint64_t shc[kScanWaves + 1];
  __shared__ uint32_t shs[kScanWaves + 1];
  const uint32_t j = blockIdx.x * kScanChunk + 4 * threadIdx.x;
  uint64_t bc = 0;  // the chunks ahead of this one
  uint32_t bs = 0;
  for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads) {
    bc += psum[i].c;
    bs += psum[i].s;
  }
  uint64_t tc, totc;
  uint32_t ts, tots;
  block_exclusive_scan<uint64_t, kScanThreads>(bc, shc, &tc);
  block_exclusive_scan<uint32_t, kScanThreads>(bs, shs, &ts);
  uint32_t c[4], k[4];
  load_chunk4(counts, cstride, caps, B, j, c, k);
  const uint64_t oc = (uint64_t)c[0] + c[1] + c[2] + c[3];
  const uint32_t os = overflow_of(c[0], k[0]) + overflow_of(c[1], k[1]) + overflow_of(c[2], k[2]) +
                      overflow_of(c[3], k[3]);
  uint64_t r = tc + block_exclusive_scan<uint64_t, kScanThreads>(oc, shc, &totc);
  uint32_t t = ts + block_exclusive_scan<uint32_t, kScanThreads>(os, shs, &tots);
  uint32_t so[4];
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    if (j + q < B) offsets[j + q] = r;
    so[q] = t;
    r += c[q];
    t += overflow_of(c[q], k[q]);
  }
  if (j + 4 <= B) {
    *reinterpret_cast<uint4*>(spill_off + j) = make_uint4(so[0], so[1], so[2], so[3]);
    if (cstride > 1) *reinterpret_cast<uint4*>(dense + j) = make_uint4(c[0], c[1], c[2], c[3]);
  } else {
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q)
      if (j + q < B) {
        spill_off[j + q] = so[q];
        if (cstride > 1) dense[j + q] = c[q];
      }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) offsets[B] = tc + totc;
}

hipError_t launch_scan_counts(uint8_t* part, const PartLayout& lay, uint32_t B, uint64_t* offsets,
                              hipStream_t st) {
  if (B >= kScanMultiMin) {
    const uint32_t g = (B + kScanChunk - 1) / kScanChunk;
    const uint32_t* pc = reinterpret_cast<const uint32_t*>(part + lay.pcounts);
    const uint32_t* caps = reinterpret_cast<const uint32_t*>(part + lay.caps);
    ScanPart* ps = reinterpret_cast<ScanPart*>(part + lay.psum);
    scan_sums_kernel<<<g, kScanThreads, 0, st>>>(pc, lay.cstride, caps, B,
                                                 reinterpret_cast<uint32_t*>(part + lay.mid_list),
                                                 reinterpret_cast<uint32_t*>(part + lay.big_list),
                                                 reinterpret_cast<PartHeader*>(part + lay.header), ps);
    scan_offsets_kernel<<<g, kScanThreads, 0, st>>>(pc, lay.cstride, reinterpret_cast<uint32_t*>(part + lay.counts),
                                                    caps, B, offsets,
                                                    reinterpret_cast<uint32_t*>(part + lay.spill_off), ps);
    return hipGetLastError();
  }
  scan_counts_kernel<<<1, kScanThreads, 0, st>>>(
      reinterpret_cast<const uint32_t*>(part + lay.pcounts), lay.cstride, reinterpret_cast<uint32_t*>(part + lay.counts),
      reinterpret_cast<const uint32_t*>(part + lay.caps), B,
      offsets, reinterpret_cast<uint32_t*>(part + lay.spill_off), reinterpret_cast<uint32_t*>(part + lay.mid_list),
      reinterpret_cast<uint32_t*>(part + lay.big_list), reinterpret_cast<PartHeader*>(part + lay.header));
  return hipGetLastError();
}

// spill_map[spill_off[b] + k] = spill slot of the k-th overflow record of bucket b.
__device__ __forceinline__ void spill_fixup_body(const PartHeader* __restrict__ ph, const uint2* __restrict__ meta,
                                                 const uint32_t* __restrict__ spill_off,
                                                 uint32_t* __restrict__ spill_map, uint32_t bid, uint32_t nblk) {
  const uint32_t m = ph->spill_count;
  for (uint32_t q = bid * 256u + threadIdx.x; q < m; q += nblk * 256u) {
    uint2 bm = meta[q];
    spill_map[spill_off[bm.x] + bm.y] = q;
  }
}

__global__ __launch_bounds__(256) void spill_fixup_kernel(const PartHeader* __restrict__ ph,
                                                          const uint2* __restrict__ meta,
                                                          const uint32_t* __restrict__ spill_off,
                                                          uint32_t* __restrict__ spill_map) {
  spill_fixup_body(ph, meta, spill_off, spill_map, blockIdx.x, gridDim.x);
}

// A window of a batch: G blocks per job.
__global__ __launch_bounds__(256) void spill_fixup_win_kernel(const WinJob* __restrict__ jobs, uint32_t G) {
  const WinJob& J = jobs[blockIdx.x / G];
  const uint8_t* part = J.part;
  spill_fixup_body(reinterpret_cast<const PartHeader*>(part + J.lay.header),
                   reinterpret_cast<const uint2*>(part + J.lay.spill_meta),
                   reinterpret_cast<const uint32_t*>(part + J.lay.spill_off),
                   reinterpret_cast<uint32_t*>(J.part + J.lay.spill_map), blockIdx.x % G, G);
}

hipError_t launch_spill_fixup_win(const WinJob* jobs, uint32_t njobs, uint32_t G, hipStream_t st) {
  if (njobs == 0 || G == 0) return hipSuccess;
  spill_fixup_win_kernel<<<njobs * G, 256, 0, st>>>(jobs, G);
  return hipGetLastError();
}

// Grid of the spill fix-up for n records.
uint32_t spill_fixup_grid(uint64_t n) {
  uint64_t g = (n + 255) / 256;
  return (uint32_t)(g > 1024 ? 1024 : (g == 0 ? 1 : g));
}

hipError_t launch_spill_fixup(uint8_t* part, const PartLayout& lay, uint64_t n, hipStream_t st) {
  spill_fixup_kernel<<<spill_fixup_grid(n), 256, 0, st>>>(reinterpret_cast<const PartHeader*>(part + lay.header),
                                           reinterpret_cast<const uint2*>(part + lay.spill_meta),
                                           reinterpret_cast<const uint32_t*>(part + lay.spill_off),
                                           reinterpret_cast<uint32_t*>(part + lay.spill_map));
  return hipGetLastError();
}

}  // namespace elsar
