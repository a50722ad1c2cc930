// Partition pass (gfx950): predict-and-place of every record (Section 3.3 and
// Algorithm 1's reader loop), the partition sizes S_p and the exclusive output
// offsets of Section 3.5, and the spill fix-up.
//
// Each block stages a tile of records in LDS with coalesced 16-byte loads,
// computes every record's base-95 code and RMI bucket, reserves a slot in the
// bucket's region with one atomic, and writes the record plus its input index
// (a 104-byte slot) with dword stores that are contiguous across lanes.  A
// bucket that outgrows its region continues in a shared spill area; the
// spill entry remembers (bucket, rank within the bucket's overflow) so the
// fix-up can group the spill without sorting it.
#include "elsar_internal.h"

namespace elsar {

constexpr int kPartThreads = 256;
constexpr int kPartTile = 256;  // records per tile (one per thread for the model step)

template <int RW_T>
__global__ __launch_bounds__(kPartThreads) void partition_kernel(
    const ModelHeader* __restrict__ hdr, const Leaf* __restrict__ leaves, const uint8_t* __restrict__ recs,
    uint64_t n, uint32_t rw_rt, uint32_t* __restrict__ counts, const uint32_t* __restrict__ caps,
    const uint32_t* __restrict__ rstart, PartHeader* __restrict__ ph, uint2* __restrict__ spill_meta,
    uint32_t* __restrict__ slots, uint64_t cap_slots) {
  const uint32_t RW = RW_T ? (uint32_t)RW_T : rw_rt;  // record dwords
  const uint32_t W = RW + 1;                           // slot dwords
  extern __shared__ uint4 tile4[];                     // kPartTile * RW dwords
  __shared__ uint32_t dst[kPartTile];
  uint32_t* tile = reinterpret_cast<uint32_t*>(tile4);
  const float a0 = hdr->a0, a1 = hdr->a1;
  const uint32_t L = hdr->L;
  const uint64_t ntiles = (n + kPartTile - 1) / kPartTile;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t r0 = t * kPartTile;
    const uint32_t cnt = (uint32_t)(n - r0 < (uint64_t)kPartTile ? n - r0 : (uint64_t)kPartTile);
    const uint32_t ndw = cnt * RW;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(recs) + r0 * RW;  // 16-byte aligned
    const uint32_t nvec = ndw >> 2;
    const uint4* src4 = reinterpret_cast<const uint4*>(src);
    for (uint32_t v = threadIdx.x; v < nvec; v += kPartThreads) tile4[v] = src4[v];
    for (uint32_t d = (nvec << 2) + threadIdx.x; d < ndw; d += kPartThreads) tile[d] = src[d];
    __syncthreads();
    if (threadIdx.x < cnt) {
      const uint32_t* r = tile + threadIdx.x * RW;
      uint64_t e = key_code(r[0], r[1]);
      uint32_t j = rmi_leaf(a0, a1, L, e);
      uint32_t b = leaf_bucket(load_leaf(leaves, j), e);
      uint32_t s = atomicAdd(&counts[b], 1u);
      uint32_t cap = caps[b];
      uint32_t slot;
      if (s < cap) {
        slot = rstart[b] + s;
      } else {
        uint32_t q = atomicAdd(&ph->spill_count, 1u);
        spill_meta[q] = make_uint2(b, s - cap);
        slot = (uint32_t)cap_slots + q;
      }
      dst[threadIdx.x] = slot;
    }
    __syncthreads();
    const uint32_t total = cnt * W;
    for (uint32_t f = threadIdx.x; f < total; f += kPartThreads) {
      uint32_t k = f / W, d = f - k * W;
      uint32_t v = d < RW ? tile[k * RW + d] : (uint32_t)(r0 + k);
      slots[(uint64_t)dst[k] * W + d] = v;
    }
    __syncthreads();
  }
}

hipError_t launch_partition(const ModelHeader* hdr, const Leaf* leaves, const uint8_t* recs, uint64_t n,
                            uint32_t rec_bytes, uint32_t /*key_bytes*/, uint8_t* part, const PartLayout& lay,
                            hipStream_t st) {
  if (n == 0) return hipSuccess;
  const uint32_t RW = rec_bytes / 4;
  const size_t lds = (size_t)kPartTile * RW * 4;
  uint64_t ntiles = (n + kPartTile - 1) / kPartTile;
  uint32_t grid = (uint32_t)(ntiles < 8192 ? ntiles : 8192);
  auto* counts = reinterpret_cast<uint32_t*>(part + lay.counts);
  auto* caps = reinterpret_cast<const uint32_t*>(part + lay.caps);
  auto* rstart = reinterpret_cast<const uint32_t*>(part + lay.rstart);
  auto* ph = reinterpret_cast<PartHeader*>(part + lay.header);
  auto* meta = reinterpret_cast<uint2*>(part + lay.spill_meta);
  auto* slots = reinterpret_cast<uint32_t*>(part + lay.slots);
  if (RW == 25)
    partition_kernel<25><<<grid, kPartThreads, lds, st>>>(hdr, leaves, recs, n, RW, counts, caps, rstart, ph, meta,
                                                          slots, lay.cap_slots);
  else
    partition_kernel<0><<<grid, kPartThreads, lds, st>>>(hdr, leaves, recs, n, RW, counts, caps, rstart, ph, meta,
                                                         slots, lay.cap_slots);
  return hipGetLastError();
}

// offsets[j] = sum_{k<j} counts[k] (u64), offsets[B] = n; spill_off[j] = sum_{k<j}
// max(counts[k] - caps[k], 0); buckets above the small LDS cap go to lists.
__global__ __launch_bounds__(1024) void scan_counts_kernel(const uint32_t* __restrict__ counts,
                                                           const uint32_t* __restrict__ caps, uint32_t B,
                                                           uint64_t* __restrict__ offsets,
                                                           uint32_t* __restrict__ spill_off,
                                                           uint32_t* __restrict__ mid_list,
                                                           uint32_t* __restrict__ big_list,
                                                           PartHeader* __restrict__ ph) {
  __shared__ uint64_t pc[1024];
  __shared__ uint32_t ps[1024];
  __shared__ uint32_t mx[1024];
  uint32_t per = (B + 1023) / 1024;
  uint32_t b = threadIdx.x * per, e = b + per < B ? b + per : B;
  uint64_t sc = 0;
  uint32_t ss = 0, m = 0;
  for (uint32_t j = b; j < e; ++j) {
    uint32_t c = counts[j], cap = caps[j];
    sc += c;
    ss += c > cap ? c - cap : 0u;
    m = c > m ? c : m;
    if (c > kSmallCap) {
      if (c <= kMidCap) mid_list[atomicAdd(&ph->n_mid, 1u)] = j;
      else big_list[atomicAdd(&ph->n_big, 1u)] = j;
    }
  }
  pc[threadIdx.x] = sc;
  ps[threadIdx.x] = ss;
  mx[threadIdx.x] = m;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint64_t x = threadIdx.x >= (unsigned)off ? pc[threadIdx.x - off] : 0ull;
    uint32_t y = threadIdx.x >= (unsigned)off ? ps[threadIdx.x - off] : 0u;
    uint32_t z = threadIdx.x >= (unsigned)off ? mx[threadIdx.x - off] : 0u;
    __syncthreads();
    pc[threadIdx.x] += x;
    ps[threadIdx.x] += y;
    mx[threadIdx.x] = z > mx[threadIdx.x] ? z : mx[threadIdx.x];
    __syncthreads();
  }
  uint64_t rc = pc[threadIdx.x] - sc;
  uint32_t rs = ps[threadIdx.x] - ss;
  for (uint32_t j = b; j < e; ++j) {
    uint32_t c = counts[j], cap = caps[j];
    offsets[j] = rc;
    spill_off[j] = rs;
    rc += c;
    rs += c > cap ? c - cap : 0u;
  }
  if (threadIdx.x == 1023) {
    offsets[B] = pc[1023];
    ph->max_count = mx[1023];
  }
}

hipError_t launch_scan_counts(uint8_t* part, const PartLayout& lay, uint32_t B, uint64_t* offsets,
                              hipStream_t st) {
  scan_counts_kernel<<<1, 1024, 0, st>>>(
      reinterpret_cast<const uint32_t*>(part + lay.counts), reinterpret_cast<const uint32_t*>(part + lay.caps), B,
      offsets, reinterpret_cast<uint32_t*>(part + lay.spill_off), reinterpret_cast<uint32_t*>(part + lay.mid_list),
      reinterpret_cast<uint32_t*>(part + lay.big_list), reinterpret_cast<PartHeader*>(part + lay.header));
  return hipGetLastError();
}

// spill_map[spill_off[b] + k] = spill slot of the k-th overflow record of bucket b.
__global__ __launch_bounds__(256) void spill_fixup_kernel(const PartHeader* __restrict__ ph,
                                                          const uint2* __restrict__ meta,
                                                          const uint32_t* __restrict__ spill_off,
                                                          uint32_t* __restrict__ spill_map) {
  const uint32_t m = ph->spill_count;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < m; q += gridDim.x * blockDim.x) {
    uint2 bm = meta[q];
    spill_map[spill_off[bm.x] + bm.y] = q;
  }
}

hipError_t launch_spill_fixup(uint8_t* part, const PartLayout& lay, uint64_t n, hipStream_t st) {
  uint32_t grid = (uint32_t)((n + 255) / 256);
  if (grid > 1024) grid = 1024;
  if (grid == 0) grid = 1;
  spill_fixup_kernel<<<grid, 256, 0, st>>>(reinterpret_cast<const PartHeader*>(part + lay.header),
                                           reinterpret_cast<const uint2*>(part + lay.spill_meta),
                                           reinterpret_cast<const uint32_t*>(part + lay.spill_off),
                                           reinterpret_cast<uint32_t*>(part + lay.spill_map));
  return hipGetLastError();
}

}  // namespace elsar
