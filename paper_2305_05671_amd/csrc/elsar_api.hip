// Host runtime of the C ABI in include/elsar.h: parameter resolution,
// workspace and partition-buffer layout, launch order and phase timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "autotune_table.h"
#include "elsar.h"
#include "elsar_internal.h"

using namespace elsar;

struct elsar_model {
  elsar_fit_params p;  // resolved parameters
  uint32_t B, L;       // buckets, leaves under the linear root
  uint32_t Lm;         // leaves under the MLP root
  uint64_t S, n;
  void* dev;           // owned allocation (null for a model placed in a workspace)
  ModelHeader* hdr;
  Leaf* leaves;
  uint32_t* hist;      // sample keys per bucket (B) under the root in use
  bool has_mlp;        // kind MLP, AUTO or SPLINE: the equi-depth state below is placed
  MlpState ms;
};

namespace {

constexpr size_t kAlign = 256;
constexpr uint32_t kDefaultMlpSteps = 16;
constexpr float kMlpLearningRate = 0.01f;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
inline bool aligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

uint64_t default_sample_size(uint64_t n) {
  uint64_t s = (n + 99) / 100;
  s = std::max<uint64_t>(s, 1024);
  s = std::min<uint64_t>(s, 10000000ull);
  return std::min<uint64_t>(s, n);
}

uint32_t default_buckets(uint64_t n) {
  uint64_t t = n / 950;
  uint32_t b = 1;
  while ((uint64_t)b * 2 <= t && b < kMaxBuckets) b *= 2;
  return b;
}

elsar_status check_params(const elsar_fit_params* p) {
  if (!p) return ELSAR_E_INVALID_ARG;
  if (p->record_bytes % 4 != 0 || p->record_bytes < 40 || p->record_bytes > 128) return ELSAR_E_UNSUPPORTED;
  if (p->key_bytes < kMinKeyBytes || p->key_bytes > kMaxKeyBytes || p->key_bytes > p->record_bytes)
    return ELSAR_E_UNSUPPORTED;
  if (p->num_buckets > kMaxBuckets) return ELSAR_E_INVALID_ARG;
  if (p->num_leaves > (1u << 22)) return ELSAR_E_INVALID_ARG;
  if (p->kind > ELSAR_MODEL_SPLINE) return ELSAR_E_INVALID_ARG;
  if (p->sample_size > 10000000ull * 4) return ELSAR_E_INVALID_ARG;
  if (p->region_pct > 1000) return ELSAR_E_INVALID_ARG;
  if (p->key_len_offset) {  // variable-length keys: the length byte sits after the key, in the first 12 bytes
    if (p->key_bytes > 11 || p->key_len_offset < p->key_bytes || p->key_len_offset > 11) return ELSAR_E_UNSUPPORTED;
  }
  return ELSAR_OK;
}

// Variable-length keys (virtual_key): the kernels' vk, and the key bytes the
// bucket sorts order (the virtual key counts its length byte).
inline uint32_t vkey(const elsar_fit_params& p) {
  return p.key_len_offset ? (p.key_len_offset << 8) | p.key_bytes : 0u;
}
inline uint32_t sort_bytes(const elsar_fit_params& p) {
  return sort_key_bytes(p.key_bytes + (p.key_len_offset ? 1u : 0u));
}

// Resolved shape of a model for n records.
struct Shape {
  uint32_t B, L, Lm;  // buckets, leaves under the linear and under the MLP root
  uint64_t S;
};

elsar_fit_params with_defaults(const elsar_fit_params& p) {
  elsar_fit_params q = p;
  if (q.region_pct == 0) q.region_pct = 125;
  if (q.accept_ratio <= 0.0f) q.accept_ratio = 1.5f;
  if (q.mlp_steps == 0) q.mlp_steps = kDefaultMlpSteps;
  return q;
}

Shape resolve(const elsar_fit_params& p, uint64_t n) {
  Shape s;
  s.B = p.num_buckets ? p.num_buckets : default_buckets(n);
  s.L = p.num_leaves ? p.num_leaves : std::max<uint32_t>(1, s.B / 16);
  // equi-depth leaves (MLP and spline roots): one per bucket by default, at
  // most 2^16 so that the routing tables (boundaries 512 KB, leaves 2 MB) stay
  // in the L2 caches
  s.Lm = p.num_leaves ? p.num_leaves : std::min<uint32_t>(s.B, 1u << 16);
  s.S = p.sample_size ? std::min<uint64_t>(p.sample_size, n) : default_sample_size(n);
  if (n > 0 && s.S == 0) s.S = 1;
  return s;
}

// Kinds with equi-depth leaves (the MLP and the spline roots).
bool wants_mlp(uint32_t kind) {
  return kind == ELSAR_MODEL_MLP || kind == ELSAR_MODEL_AUTO || kind == ELSAR_MODEL_SPLINE;
}

size_t model_dev_bytes(const Shape& sh, uint32_t kind) {
  size_t b = align_up(sizeof(ModelHeader)) + align_up((size_t)sh.L * sizeof(Leaf)) + align_up((size_t)sh.B * 4);
  if (wants_mlp(kind)) b += align_up(mlp_state_bytes(sh.Lm, sh.B));
  return b;
}

void place_model(elsar_model* m, void* base) {
  uint8_t* b = static_cast<uint8_t*>(base);
  m->hdr = reinterpret_cast<ModelHeader*>(b);
  b += align_up(sizeof(ModelHeader));
  m->leaves = reinterpret_cast<Leaf*>(b);
  b += align_up((size_t)m->L * sizeof(Leaf));
  m->hist = reinterpret_cast<uint32_t*>(b);
  b += align_up((size_t)m->B * 4);
  m->has_mlp = wants_mlp(m->p.kind);
  m->ms = MlpState{};
  if (m->has_mlp) place_mlp_state(&m->ms, b, m->Lm, m->B);
}

size_t fit_ws_bytes(uint64_t S) {
  return 2 * align_up((size_t)S * 8) + align_up(radix_u64_scratch_bytes(S)) + align_up(fit_scratch_bytes(S));
}

PartLayout part_layout(uint64_t n, uint32_t B, uint32_t R, uint32_t region_pct, uint32_t K) {
  PartLayout lay{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  lay.header = take(sizeof(PartHeader));
  lay.counts = take((size_t)B * 4);
  lay.cstride = counter_stride(B);
  lay.pcounts = lay.cstride > 1 ? take((size_t)B * lay.cstride * 4) : lay.counts;
  lay.caps = take((size_t)B * 4);
  lay.rstart = take((size_t)B * 4);
  lay.spill_off = take((size_t)B * 4);
  lay.mid_list = take((size_t)B * 4);
  lay.big_list = take((size_t)B * 4);
  lay.big2_list = take((size_t)B * 4);
  lay.psum = take((size_t)(B + kScanChunk - 1) / kScanChunk * sizeof(ScanPart));
  lay.spill_meta = take((size_t)n * 8);
  lay.spill_map = take((size_t)n * 4);
  // split of buckets above the LDS caps: every split of c entries gives at most
  // 3c / 2048 + 1 segments, one split per composite byte and level
  lay.seg_leaf_cap = (uint32_t)std::min<uint64_t>(n / 32 + 4096, 0xFFFFFFFFull);
  lay.seg_leaf = take((size_t)lay.seg_leaf_cap * 16);
  // regions: sum_j ceil(f * max(n h_j / S, n / B)) + 17 <= 2 f n + 18 B,  f = region_pct / 100
  lay.cap_slots = (n * 2 * region_pct + 99) / 100 + 18ull * B + 16;
  lay.total_slots = lay.cap_slots + n;
  lay.slot_bytes = slot_bytes_for(R);
  // after the bucket sorts the slot area is the scratch of the long-key fix-up
  size_t slot_area = (size_t)lay.total_slots * lay.slot_bytes;
  if (K > kSortKeyBytes) slot_area = std::max(slot_area, long_key_scratch_bytes(n, R));
  lay.slots = take(slot_area);
  lay.bytes = off;
  return lay;
}

// ------------------------------------------------------------ phase timing --
constexpr int kTimedPhases = 6;  // boundaries: start, fit, partition, scan, LDS sort, all bucket kernels
constexpr int kTimingSlots = 512;

struct Timing {
  std::mutex mu;
  bool on = false;
  std::vector<hipEvent_t> ev;  // kTimingSlots * kTimedPhases
  std::vector<uint8_t> have;   // which boundaries of a slot were recorded
  int next = 0, used = 0;
} g_timing;

struct PhaseMarks {  // events of the current call, or nulls when timing is off
  hipEvent_t e[kTimedPhases] = {};
  int slot = -1;
};

PhaseMarks begin_marks() {
  PhaseMarks pm;
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (!g_timing.on) return pm;
  pm.slot = g_timing.next;
  g_timing.next = (g_timing.next + 1) % kTimingSlots;
  g_timing.used = std::min(g_timing.used + 1, kTimingSlots);
  g_timing.have[pm.slot] = 0;
  for (int i = 0; i < kTimedPhases; ++i) pm.e[i] = g_timing.ev[pm.slot * kTimedPhases + i];
  return pm;
}

void mark(PhaseMarks& pm, int i, hipStream_t st) {
  if (pm.slot < 0) return;
  if (hipEventRecord(pm.e[i], st) == hipSuccess) g_timing.have[pm.slot] |= (uint8_t)(1u << i);
}

#define HIP_TRY(x)                                  \
  do {                                              \
    if ((x) != hipSuccess) return ELSAR_E_HIP;      \
  } while (0)

// --------------------------------------------------------------- pipeline --
elsar_status do_fit(elsar_model* m, const void* d_records, uint64_t n, void* d_ws, size_t ws_bytes,
                    hipStream_t st) {
  if (n == 0) return ELSAR_OK;
  const uint64_t S = m->S;
  if (ws_bytes < fit_ws_bytes(S)) return ELSAR_E_NO_MEMORY;
  uint8_t* w = static_cast<uint8_t*>(d_ws);
  uint64_t* codes = reinterpret_cast<uint64_t*>(w);
  uint64_t* tmp = reinterpret_cast<uint64_t*>(w + align_up(S * 8));
  void* rscr = w + 2 * align_up(S * 8);
  void* fscr = w + 2 * align_up(S * 8) + align_up(radix_u64_scratch_bytes(S));
  HIP_TRY(launch_sample_codes(static_cast<const uint8_t*>(d_records), n, m->p.record_bytes, S, m->p.seed, codes,
                              st, vkey(m->p)));
  if (m->p.kind == ELSAR_MODEL_RADIX) {  // equi-width buckets; the sample only sizes the regions
    HIP_TRY(launch_radix_model(S, n, m->L, m->B, m->hdr, m->leaves, st));
    HIP_TRY(launch_sample_hist(m->hdr, m->leaves, codes, S, m->B, m->hist, st));
    HIP_TRY(launch_decide_root(m->hist, nullptr, m->B, S, m->p.accept_ratio, m->p.kind, m->hdr, m->hist, st));
    m->n = n;
    return ELSAR_OK;
  }
  uint64_t* sorted = nullptr;
  // codes < 95^8 < 2^53: bytes 0..6 carry the value
  HIP_TRY(launch_radix_sort_u64(codes, tmp, S, 0, 6, rscr, st, &sorted));
  HIP_TRY(launch_fit_rmi(sorted, S, n, m->L, m->B, m->hdr, m->leaves, fscr, st));
  HIP_TRY(launch_sample_hist(m->hdr, m->leaves, sorted, S, m->B, m->hist, st));
  if (m->has_mlp) {
    HIP_TRY(launch_auto_gate(m->hist, m->B, S, m->p.accept_ratio, m->p.kind, m->hdr, st));
    if (m->p.kind == ELSAR_MODEL_MLP) {
      const uint32_t steps = m->p.mlp_steps == ELSAR_MLP_STEPS_NONE ? 0u : m->p.mlp_steps;
      HIP_TRY(launch_mlp_train(sorted, S, m->p.seed, steps, kMlpLearningRate, m->ms, st));
    }
    HIP_TRY(launch_equi_depth_leaves(sorted, S, m->Lm, m->B, m->hdr, m->ms, st));
    if (m->p.kind == ELSAR_MODEL_MLP) {
      HIP_TRY(launch_mlp_net_hist(m->ms, sorted, S, m->B, st));
    }
  }
  HIP_TRY(launch_decide_root(m->hist, m->has_mlp ? &m->ms : nullptr, m->B, S, m->p.accept_ratio, m->p.kind,
                             m->hdr, m->hist, st));
  if (m->has_mlp && m->p.kind == ELSAR_MODEL_MLP) HIP_TRY(launch_mlp_cell_table(m->ms, m->Lm, m->hdr, st));
  m->n = n;
  return ELSAR_OK;
}

elsar_status do_partition(const elsar_model* m, const void* d_records, uint64_t n, void* d_part,
                          size_t part_bytes, uint64_t* d_offsets, hipStream_t st, PhaseMarks* pm) {
  PartLayout lay = part_layout(n, m->B, m->p.record_bytes, m->p.region_pct, m->p.key_bytes);
  if (lay.total_slots >= (1ull << 32)) return ELSAR_E_UNSUPPORTED;  // slot indices are 32-bit
  if (part_bytes < lay.bytes) return ELSAR_E_NO_MEMORY;
  uint8_t* part = static_cast<uint8_t*>(d_part);
  HIP_TRY(launch_capacities(m->hist, m->S, n, m->B, m->p.region_pct, part, lay, st));
  if (pm) mark(*pm, 1, st);
  HIP_TRY(launch_partition(m->hdr, m->leaves, m->has_mlp ? &m->ms : nullptr, static_cast<const uint8_t*>(d_records),
                           n, m->p.record_bytes, vkey(m->p), part, lay, st));
  if (pm) mark(*pm, 2, st);
  HIP_TRY(launch_scan_counts(part, lay, m->B, d_offsets, st));
  HIP_TRY(launch_spill_fixup(part, lay, n, st));
  return ELSAR_OK;
}

elsar_status do_sort_buckets(const elsar_model* m, void* d_part, size_t part_bytes, uint64_t n,
                             const uint64_t* d_offsets, void* d_out, hipStream_t st, PhaseMarks* pm) {
  PartLayout lay = part_layout(n, m->B, m->p.record_bytes, m->p.region_pct, m->p.key_bytes);
  if (part_bytes < lay.bytes) return ELSAR_E_NO_MEMORY;
  uint8_t* part = static_cast<uint8_t*>(d_part);
  uint8_t* out = static_cast<uint8_t*>(d_out);
  const uint32_t K = m->p.key_bytes, Ks = sort_bytes(m->p), vk = vkey(m->p);
  HIP_TRY(launch_bucket_sort_small(part, lay, m->B, d_offsets, m->p.record_bytes, Ks, out, st, vk));
  if (pm) mark(*pm, 4, st);
  HIP_TRY(launch_bucket_sort_large(part, lay, m->B, n, d_offsets, m->p.record_bytes, Ks, out, st, vk));
  HIP_TRY(launch_long_key_fixup(out, n, m->p.record_bytes, K, part + lay.slots, st));
  if (pm) mark(*pm, 5, st);
  return ELSAR_OK;
}

struct SortLayout {
  size_t model, fit, part, offsets, bytes;
  PartLayout lay;
};

SortLayout sort_layout(const elsar_fit_params& p, const Shape& sh, uint64_t n) {
  SortLayout sl{};
  size_t off = 0;
  sl.model = off;
  off += align_up(model_dev_bytes(sh, p.kind));
  sl.fit = off;
  off += align_up(fit_ws_bytes(sh.S));
  sl.offsets = off;
  off += align_up(((size_t)sh.B + 1) * 8);
  sl.lay = part_layout(n, sh.B, p.record_bytes, p.region_pct, p.key_bytes);
  sl.part = off;
  off += align_up(sl.lay.bytes);
  sl.bytes = off;
  return sl;
}

}  // namespace

// ====================================================================== ABI ==
extern "C" {

elsar_status elsar_fit_params_default(elsar_fit_params* p) {
  if (!p) return ELSAR_E_INVALID_ARG;
  std::memset(p, 0, sizeof(*p));
  p->record_bytes = 100;
  p->key_bytes = 10;
  p->kind = ELSAR_MODEL_RMI;
  p->accept_ratio = 1.5f;
  return ELSAR_OK;
}

elsar_status elsar_model_create(const elsar_fit_params* p, uint64_t n, elsar_model** out) {
  if (!out) return ELSAR_E_INVALID_ARG;
  *out = nullptr;
  elsar_status s = check_params(p);
  if (s != ELSAR_OK) return s;
  if (n > ELSAR_MAX_DEVICE_RECORDS) return ELSAR_E_UNSUPPORTED;
  Shape sh = resolve(*p, n);
  elsar_model* m = new (std::nothrow) elsar_model();
  if (!m) return ELSAR_E_NO_MEMORY;
  m->p = with_defaults(*p);
  m->B = sh.B;
  m->L = sh.L;
  m->Lm = sh.Lm;
  m->S = sh.S;
  m->n = 0;
  if (hipMalloc(&m->dev, model_dev_bytes(sh, m->p.kind)) != hipSuccess) {
    delete m;
    return ELSAR_E_NO_MEMORY;
  }
  place_model(m, m->dev);
  *out = m;
  return ELSAR_OK;
}

void elsar_model_destroy(elsar_model* m) {
  if (!m) return;
  if (m->dev) (void)hipFree(m->dev);
  delete m;
}

elsar_status elsar_fit_workspace_size(const elsar_model* m, uint64_t /*n*/, size_t* bytes) {
  if (!m || !bytes) return ELSAR_E_INVALID_ARG;
  *bytes = fit_ws_bytes(m->S);
  return ELSAR_OK;
}

elsar_status elsar_sample_fit(elsar_model* m, const void* d_records, uint64_t n, void* d_ws, size_t ws_bytes,
                              hipStream_t stream) {
  if (!m) return ELSAR_E_INVALID_ARG;
  if (n > ELSAR_MAX_DEVICE_RECORDS) return ELSAR_E_UNSUPPORTED;
  if (n && (!d_records || !d_ws || !aligned16(d_records))) return ELSAR_E_INVALID_ARG;
  Shape sh = resolve(m->p, n);
  if (sh.B != m->B || sh.L != m->L || sh.Lm != m->Lm) return ELSAR_E_INVALID_ARG;  // model shaped for another n
  m->S = sh.S;
  if (ws_bytes < fit_ws_bytes(m->S)) return ELSAR_E_NO_MEMORY;
  elsar_status s = do_fit(m, d_records, n, d_ws, ws_bytes, stream);
  if (s != ELSAR_OK || m->p.kind != ELSAR_MODEL_MLP || n == 0) return s;
  ModelHeader h;
  HIP_TRY(hipMemcpyAsync(&h, m->hdr, sizeof(h), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return h.kind_used == 1 ? ELSAR_OK : ELSAR_E_MODEL_REJECTED;
}

elsar_status elsar_partition_size(const elsar_model* m, uint64_t n, size_t* part_bytes) {
  if (!m || !part_bytes) return ELSAR_E_INVALID_ARG;
  if (n > ELSAR_MAX_DEVICE_RECORDS) return ELSAR_E_UNSUPPORTED;
  *part_bytes = part_layout(n, m->B, m->p.record_bytes, m->p.region_pct, m->p.key_bytes).bytes;
  return ELSAR_OK;
}

elsar_status elsar_partition(const elsar_model* m, const void* d_records, uint64_t n, void* d_part,
                             size_t part_bytes, uint64_t* d_bucket_offsets, hipStream_t stream) {
  if (!m || !d_part || !d_bucket_offsets) return ELSAR_E_INVALID_ARG;
  if (!aligned16(d_part) || !aligned8(d_bucket_offsets)) return ELSAR_E_INVALID_ARG;
  if (n > ELSAR_MAX_DEVICE_RECORDS) return ELSAR_E_UNSUPPORTED;
  if (n && (!d_records || !aligned16(d_records))) return ELSAR_E_INVALID_ARG;
  if (m->n == 0 && n > 0) return ELSAR_E_INVALID_ARG;  // not fitted
  PhaseMarks pm = begin_marks();
  mark(pm, 0, stream);
  elsar_status s = do_partition(m, d_records, n, d_part, part_bytes, d_bucket_offsets, stream, &pm);
  mark(pm, 3, stream);
  return s;
}

elsar_status elsar_sort_buckets(const elsar_model* m, void* d_part, size_t part_bytes, uint64_t n,
                                const uint64_t* d_bucket_offsets, void* d_out, hipStream_t stream) {
  if (!m || !d_part || !d_bucket_offsets) return ELSAR_E_INVALID_ARG;
  if (!aligned16(d_part) || !aligned8(d_bucket_offsets)) return ELSAR_E_INVALID_ARG;
  if (n > ELSAR_MAX_DEVICE_RECORDS) return ELSAR_E_UNSUPPORTED;
  if (n && (!d_out || !aligned16(d_out))) return ELSAR_E_INVALID_ARG;
  PhaseMarks pm = begin_marks();
  mark(pm, 3, stream);
  return do_sort_buckets(m, d_part, part_bytes, n, d_bucket_offsets, d_out, stream, &pm);
}

elsar_status elsar_sort_workspace_size(const elsar_fit_params* p, uint64_t n, size_t* bytes) {
  if (!bytes) return ELSAR_E_INVALID_ARG;
  elsar_status s = check_params(p);
  if (s != ELSAR_OK) return s;
  if (n > ELSAR_MAX_DEVICE_RECORDS) return ELSAR_E_UNSUPPORTED;
  elsar_fit_params q = with_defaults(*p);
  *bytes = sort_layout(q, resolve(q, n), n).bytes;
  return ELSAR_OK;
}

}  // extern "C"

namespace {

// One whole sort on device-resident records; q has its defaults filled in.
elsar_status sort_job(const void* d_in, uint64_t n, void* d_out, const elsar_fit_params& q, void* d_ws,
                      size_t ws_bytes, hipStream_t stream, bool timed) {
  Shape sh = resolve(q, n);
  SortLayout sl = sort_layout(q, sh, n);
  if (ws_bytes < sl.bytes) return ELSAR_E_NO_MEMORY;
  if (n == 1) {
    if (d_out != d_in) HIP_TRY(hipMemcpyAsync(d_out, d_in, q.record_bytes, hipMemcpyDeviceToDevice, stream));
    return ELSAR_OK;
  }
  uint8_t* w = static_cast<uint8_t*>(d_ws);
  elsar_model m{};
  m.p = q;
  m.B = sh.B;
  m.L = sh.L;
  m.Lm = sh.Lm;
  m.S = sh.S;
  m.dev = nullptr;
  place_model(&m, w + sl.model);
  uint64_t* offsets = reinterpret_cast<uint64_t*>(w + sl.offsets);
  PhaseMarks pm = timed ? begin_marks() : PhaseMarks{};
  mark(pm, 0, stream);
  elsar_status s = do_fit(&m, d_in, n, w + sl.fit, fit_ws_bytes(sh.S), stream);
  if (s != ELSAR_OK) return s;
  s = do_partition(&m, d_in, n, w + sl.part, sl.lay.bytes, offsets, stream, &pm);
  if (s != ELSAR_OK) return s;
  mark(pm, 3, stream);
  return do_sort_buckets(&m, w + sl.part, sl.lay.bytes, n, offsets, d_out, stream, &pm);
}

// ------------------------------------------------------------------ batch --
constexpr uint32_t kBatchLanes = 16;
constexpr size_t kMaxPlans = 8;

uint32_t ceil_log2(uint64_t n) {
  uint32_t r = 0;
  while ((1ull << r) < n) ++r;
  return r;
}

uint32_t tuned_buckets(uint64_t n) {
  const uint32_t r = ceil_log2(n);
  const uint32_t per = r < kAutotuneRows ? kAutotuneRecordsPerBucket[r] : 0u;
  if (per == 0) return default_buckets(n);
  uint32_t b = 1;
  while ((uint64_t)b * 2 * per <= n && b < kMaxBuckets) b *= 2;
  return b;
}

elsar_fit_params job_params(const elsar_fit_params& p, uint64_t n, uint32_t j) {
  elsar_fit_params q = p;
  if (q.num_buckets == 0) q.num_buckets = tuned_buckets(n);
  q.seed = p.seed + j;
  return with_defaults(q);
}

// A window: jobs whose sizes differ by at most 2x and whose partition buffers
// fit the window area together, sorted by one launch per phase.
struct BatchWindow {
  std::vector<uint32_t> jobs;  // job indices, largest first
  uint64_t nmax = 0;           // records of its largest job
  uint32_t Bmax = 0;           // buckets of its job with the most
  bool prefit_only = true;     // every model comes from the batched fit kernel
  size_t desc = 0;             // workspace offset of its WinJob array
};

struct BatchLayout {
  std::vector<TinyJob> tiny;
  std::vector<uint32_t> prefit;                  // jobs whose model the batch fit kernel fits
  std::vector<size_t> prefit_scratch;            // per such job: offset of its sample scratch (larger samples)
  std::vector<size_t> model;                     // per job above kSmallCap: workspace offset of its model
  std::vector<std::vector<uint32_t>> fit_lanes;  // the other jobs, fitted one by one, per lane
  std::vector<size_t> fit_off, fit_bytes;        // per lane: its fit scratch
  std::vector<BatchWindow> windows;              // smallest jobs first
  size_t fit_desc = 0, tiny_desc = 0, tiny_stage = 0, win_desc = 0, area = 0, area_bytes = 0, bytes = 0;
};

// Records per window, unless one job alone is larger: about the 100M-record
// sort's working set (a window of this many records needs about 30 GB of
// partition buffers), large enough that every phase kernel fills the GPU.
constexpr uint64_t kWindowRecords = 64ull << 20;

// Window-area bytes of one job: its B + 1 output offsets, then its partition buffer.
size_t window_job_bytes(const elsar_fit_params& q, const Shape& sh, uint64_t n) {
  return align_up(((size_t)sh.B + 1) * 8) +
         align_up(part_layout(n, sh.B, q.record_bytes, q.region_pct, q.key_bytes).bytes);
}

elsar_status batch_layout(const elsar_job* jobs, uint32_t njobs, const elsar_fit_params& p, BatchLayout* bl) {
  const uint32_t RW = p.record_bytes / 4;
  std::vector<uint32_t> big;
  uint64_t stage_dw = 0;
  for (uint32_t j = 0; j < njobs; ++j) {
    const elsar_job& J = jobs[j];
    if (J.n == 0) continue;
    if (J.n > ELSAR_MAX_DEVICE_RECORDS) return ELSAR_E_UNSUPPORTED;
    if (!J.d_in || !J.d_out || !aligned16(J.d_in) || !aligned16(J.d_out)) return ELSAR_E_INVALID_ARG;
    if (J.n <= kSmallCap) {
      TinyJob t{};
      t.in = static_cast<const uint32_t*>(J.d_in);
      t.out = static_cast<uint32_t*>(J.d_out);
      t.n = (uint32_t)J.n;
      t.staging_dw = stage_dw;
      if (J.d_in == J.d_out) stage_dw += (J.n * RW + 3) & ~3ull;
      bl->tiny.push_back(t);
    } else {
      const elsar_fit_params q = job_params(p, J.n, j);
      if (part_layout(J.n, resolve(q, J.n).B, q.record_bytes, q.region_pct, q.key_bytes).total_slots >= (1ull << 32))
        return ELSAR_E_UNSUPPORTED;  // slot indices are 32-bit
      big.push_back(j);
    }
  }
  std::stable_sort(big.begin(), big.end(), [&](uint32_t a, uint32_t b) { return jobs[a].n > jobs[b].n; });
  // models: one batched kernel for the linear root of jobs whose sample it
  // can sort; the others one by one, longest sample first to the least loaded
  // lane
  std::vector<uint8_t> is_prefit(njobs, 0);
  std::vector<uint32_t> lone;
  for (uint32_t j : big) {
    const elsar_fit_params q = job_params(p, jobs[j].n, j);
    if (p.kind == ELSAR_MODEL_RMI && resolve(q, jobs[j].n).S <= kBatchFitMaxS * kBatchFitChunks) {
      bl->prefit.push_back(j);
      is_prefit[j] = 1;
    } else {
      lone.push_back(j);
    }
  }
  const uint32_t nl = std::min<uint32_t>(kBatchLanes, (uint32_t)lone.size());
  bl->fit_lanes.assign(nl, {});
  bl->fit_bytes.assign(nl, 0);
  std::vector<uint64_t> load(nl, 0);
  for (uint32_t j : lone) {
    const uint32_t l = (uint32_t)(std::min_element(load.begin(), load.end()) - load.begin());
    const uint64_t S = resolve(job_params(p, jobs[j].n, j), jobs[j].n).S;
    bl->fit_lanes[l].push_back(j);
    load[l] += S;
    bl->fit_bytes[l] = std::max(bl->fit_bytes[l], fit_ws_bytes(S));
  }
  // windows over the jobs in decreasing size: a window takes jobs while they
  // are at least half its largest and fit its record budget
  for (size_t i = 0; i < big.size();) {
    BatchWindow w;
    w.nmax = jobs[big[i]].n;
    const uint64_t budget = std::max<uint64_t>(kWindowRecords, w.nmax);
    uint64_t sum = 0;
    while (i < big.size()) {
      const uint32_t j = big[i];
      const uint64_t n = jobs[j].n;
      const uint32_t B = resolve(job_params(p, n, j), n).B;
      const uint64_t most = std::max<uint64_t>(std::max(B, w.Bmax), 2048);  // largest per-job grid
      if (!w.jobs.empty() && (2 * n < w.nmax || sum + n > budget || (w.jobs.size() + 1) * most > 0x7FFFFFFFull))
        break;
      w.jobs.push_back(j);
      w.Bmax = std::max(w.Bmax, B);
      w.prefit_only = w.prefit_only && is_prefit[j];
      sum += n;
      ++i;
    }
    bl->windows.push_back(std::move(w));
  }
  std::reverse(bl->windows.begin(), bl->windows.end());
  size_t off = 0;
  bl->tiny_desc = off;
  off += align_up(bl->tiny.size() * sizeof(TinyJob));
  bl->fit_desc = off;
  off += align_up(bl->prefit.size() * sizeof(FitJob));
  bl->model.assign(njobs, 0);
  for (uint32_t j : big) {
    const elsar_fit_params q = job_params(p, jobs[j].n, j);
    bl->model[j] = off;
    off += align_up(model_dev_bytes(resolve(q, jobs[j].n), q.kind));
  }
  for (uint32_t j : bl->prefit) {
    const uint64_t S = resolve(job_params(p, jobs[j].n, j), jobs[j].n).S;
    bl->prefit_scratch.push_back(S > kBatchFitMaxS ? off : 0);
    if (S > kBatchFitMaxS) off += align_up((size_t)S * 16);
  }
  bl->tiny_stage = off;
  off += align_up(stage_dw * 4);
  bl->fit_off.assign(nl, 0);
  for (uint32_t l = 0; l < nl; ++l) {
    bl->fit_off[l] = off;
    off += align_up(bl->fit_bytes[l]);
  }
  bl->win_desc = off;  // every window's WinJob array, one after another
  off += align_up(big.size() * sizeof(WinJob));
  size_t k = 0;
  for (BatchWindow& w : bl->windows) {
    w.desc = bl->win_desc + k * sizeof(WinJob);
    k += w.jobs.size();
    size_t a = 0;
    for (uint32_t j : w.jobs) {
      const elsar_fit_params q = job_params(p, jobs[j].n, j);
      a += window_job_bytes(q, resolve(q, jobs[j].n), jobs[j].n);
    }
    bl->area_bytes = std::max(bl->area_bytes, a);
  }
  bl->area = off;
  off += bl->area_bytes;
  bl->bytes = std::max<size_t>(off, 256);
  return ELSAR_OK;
}

// A job's model, placed where the layout keeps it.
elsar_model job_model(const elsar_job* jobs, const elsar_fit_params& p, const BatchLayout& bl, uint8_t* w,
                      uint32_t j) {
  const elsar_fit_params q = job_params(p, jobs[j].n, j);
  const Shape sh = resolve(q, jobs[j].n);
  elsar_model m{};
  m.p = q;
  m.B = sh.B;
  m.L = sh.L;
  m.Lm = sh.Lm;
  m.S = sh.S;
  place_model(&m, w + bl.model[j]);
  return m;
}

std::vector<FitJob> fit_descriptors(const elsar_job* jobs, const elsar_fit_params& p, const BatchLayout& bl,
                                    uint8_t* w) {
  std::vector<FitJob> out;
  for (size_t k = 0; k < bl.prefit.size(); ++k) {
    const uint32_t j = bl.prefit[k];
    const elsar_model m = job_model(jobs, p, bl, w, j);
    FitJob f{};
    f.scratch = bl.prefit_scratch[k] ? reinterpret_cast<uint64_t*>(w + bl.prefit_scratch[k]) : nullptr;
    f.recs = static_cast<const uint8_t*>(jobs[j].d_in);
    f.n = jobs[j].n;
    f.S = m.S;
    f.seed = m.p.seed;
    f.L = m.L;
    f.B = m.B;
    f.hdr = m.hdr;
    f.leaves = m.leaves;
    f.hist = m.hist;
    out.push_back(f);
  }
  return out;
}

// The WinJob arrays of every window, in window order.
std::vector<WinJob> window_descriptors(const elsar_job* jobs, const elsar_fit_params& p, const BatchLayout& bl,
                                       uint8_t* w) {
  std::vector<WinJob> out;
  for (const BatchWindow& win : bl.windows) {
    size_t a = bl.area;
    for (uint32_t j : win.jobs) {
      const elsar_model m = job_model(jobs, p, bl, w, j);
      WinJob J{};
      J.recs = static_cast<const uint8_t*>(jobs[j].d_in);
      J.out = static_cast<uint8_t*>(jobs[j].d_out);
      J.n = jobs[j].n;
      J.S = m.S;
      J.hdr = m.hdr;
      J.leaves = m.leaves;
      J.hist = m.hist;
      if (m.has_mlp) {
        J.mlp = m.ms.M;
        J.eq_leaves = m.ms.leaves;
        J.bound = m.ms.bound;
        J.ccells = m.ms.ccells;
        J.cells = m.ms.cells;
      }
      J.offsets = reinterpret_cast<uint64_t*>(w + a);
      J.lay = part_layout(J.n, m.B, m.p.record_bytes, m.p.region_pct, m.p.key_bytes);
      J.part = w + a + align_up(((size_t)m.B + 1) * 8);
      J.B = m.B;
      a += window_job_bytes(m.p, resolve(m.p, J.n), J.n);
      out.push_back(J);
    }
  }
  return out;
}

struct BatchPlan {
  std::vector<uint8_t> key;
  std::vector<FitJob> fit;    // sources of the per-launch descriptor uploads
  std::vector<TinyJob> tiny;
  std::vector<WinJob> win;    // every window's jobs, in window order
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

std::mutex g_batch_mu;
std::list<BatchPlan> g_plans;  // most recently used first

std::vector<uint8_t> plan_key(const elsar_job* jobs, uint32_t njobs, const elsar_fit_params& p, const void* ws,
                              size_t ws_bytes) {
  std::vector<uint8_t> k(sizeof(elsar_fit_params) + sizeof(void*) + sizeof(size_t) + (size_t)njobs * sizeof(elsar_job));
  uint8_t* o = k.data();
  std::memcpy(o, &p, sizeof(p));
  o += sizeof(p);
  std::memcpy(o, &ws, sizeof(ws));
  o += sizeof(ws);
  std::memcpy(o, &ws_bytes, sizeof(ws_bytes));
  o += sizeof(ws_bytes);
  if (njobs) std::memcpy(o, jobs, (size_t)njobs * sizeof(elsar_job));
  return k;
}

// One window: each phase one launch over all its jobs.
elsar_status enqueue_window(const BatchWindow& win, const elsar_fit_params& p, uint8_t* w, hipStream_t st) {
  const WinJob* d = reinterpret_cast<const WinJob*>(w + win.desc);
  const uint32_t nj = (uint32_t)win.jobs.size();
  const uint32_t row = ceil_log2(win.nmax);
  const WinGrids g = window_grids(win.nmax, win.Bmax, row < kAutotuneRows ? kAutotunePartTilesPerBlock[row] : 0u);
  const elsar_fit_params q = with_defaults(p);
  HIP_TRY(launch_capacities_win(d, nj, q.region_pct, st));
  HIP_TRY(launch_partition_win(d, nj, g.part, q.record_bytes, wants_mlp(q.kind), st));
  HIP_TRY(launch_scan_counts_win(d, nj, st));
  HIP_TRY(launch_spill_fixup_win(d, nj, g.fixup, st));
  HIP_TRY(launch_bucket_sort_small_win(d, nj, g.small, q.record_bytes, sort_bytes(q), st));
  HIP_TRY(launch_bucket_sort_large_win(d, nj, g, q.record_bytes, sort_bytes(q), st));
  return ELSAR_OK;
}

// Every kernel of the batch: the small jobs, the batched fit and the windows
// on `cap`; the models fitted one by one on lane streams forked from it, beside
// the windows whose models the batched fit provides, and joined back before the
// first window that needs them.
elsar_status enqueue_batch(const elsar_job* jobs, const elsar_fit_params& p, const BatchLayout& bl, uint8_t* w,
                           hipStream_t cap, hipStream_t* lanes, hipEvent_t fork, hipEvent_t* done) {
  const size_t nl = bl.fit_lanes.size();
  if (nl) {
    HIP_TRY(hipEventRecord(fork, cap));
    for (size_t l = 0; l < nl; ++l) {
      HIP_TRY(hipStreamWaitEvent(lanes[l], fork, 0));
      for (uint32_t j : bl.fit_lanes[l]) {
        elsar_model m = job_model(jobs, p, bl, w, j);
        elsar_status s = do_fit(&m, jobs[j].d_in, jobs[j].n, w + bl.fit_off[l], bl.fit_bytes[l], lanes[l]);
        if (s != ELSAR_OK) return s;
      }
      HIP_TRY(hipEventRecord(done[l], lanes[l]));
    }
  }
  if (!bl.tiny.empty())
    HIP_TRY(launch_tiny_jobs(reinterpret_cast<const TinyJob*>(w + bl.tiny_desc), (uint32_t)bl.tiny.size(),
                             p.record_bytes, p.key_bytes, reinterpret_cast<uint32_t*>(w + bl.tiny_stage), cap));
  if (!bl.prefit.empty())
    HIP_TRY(launch_batch_fit(reinterpret_cast<const FitJob*>(w + bl.fit_desc), (uint32_t)bl.prefit.size(),
                             p.record_bytes, cap));
  bool joined = nl == 0;
  auto join = [&]() -> elsar_status {
    for (size_t l = 0; l < nl; ++l) HIP_TRY(hipStreamWaitEvent(cap, done[l], 0));
    joined = true;
    return ELSAR_OK;
  };
  for (const BatchWindow& win : bl.windows) {
    if (!joined && !win.prefit_only) {
      elsar_status s = join();
      if (s != ELSAR_OK) return s;
    }
    elsar_status s = enqueue_window(win, p, w, cap);
    if (s != ELSAR_OK) return s;
  }
  return joined ? ELSAR_OK : join();
}

elsar_status build_plan(const elsar_job* jobs, const elsar_fit_params& p, const BatchLayout& bl, uint8_t* w,
                        BatchPlan* plan) {
  hipStream_t cap = nullptr, lanes[kBatchLanes] = {};
  hipEvent_t fork = nullptr, done[kBatchLanes] = {};
  elsar_status s = ELSAR_OK;
  auto cleanup = [&]() {
    if (cap) (void)hipStreamDestroy(cap);
    for (auto& x : lanes)
      if (x) (void)hipStreamDestroy(x);
    if (fork) (void)hipEventDestroy(fork);
    for (auto& e : done)
      if (e) (void)hipEventDestroy(e);
  };
  if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) {
    cleanup();
    return ELSAR_E_HIP;
  }
  for (uint32_t l = 0; l < kBatchLanes; ++l)
    if (hipStreamCreateWithFlags(&lanes[l], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&done[l], hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return ELSAR_E_HIP;
    }
  if (p.kind != ELSAR_MODEL_RMI && mlp_prepare_kernels() != hipSuccess) {
    cleanup();
    return ELSAR_E_HIP;
  }
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    cleanup();
    return ELSAR_E_HIP;
  }
  s = enqueue_batch(jobs, p, bl, w, cap, lanes, fork, done);
  hipGraph_t g = nullptr;
  const hipError_t ec = hipStreamEndCapture(cap, &g);
  if (s == ELSAR_OK && ec != hipSuccess) s = ELSAR_E_HIP;
  if (s == ELSAR_OK && hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0) != hipSuccess) s = ELSAR_E_HIP;
  if (s != ELSAR_OK) {
    if (g) (void)hipGraphDestroy(g);
    plan->exec = nullptr;
  } else {
    plan->graph = g;
  }
  cleanup();
  return s;
}

}  // namespace

extern "C" {

elsar_status elsar_sort(const void* d_in, uint64_t n, void* d_out, const elsar_fit_params* p, void* d_ws,
                        size_t ws_bytes, hipStream_t stream) {
  elsar_status s = check_params(p);
  if (s != ELSAR_OK) return s;
  if (n > ELSAR_MAX_DEVICE_RECORDS) return ELSAR_E_UNSUPPORTED;
  if (n == 0) return ELSAR_OK;
  if (!d_in || !d_out || !d_ws || !aligned16(d_in) || !aligned16(d_out) || !aligned16(d_ws))
    return ELSAR_E_INVALID_ARG;
  return sort_job(d_in, n, d_out, with_defaults(*p), d_ws, ws_bytes, stream, true);
}

}  // extern "C"

// --------------------------------------------------- no-allocation entry --
// The workspace of elsar_sort_noalloc: one array per device, in the code
// object, held until the process ends.  Host code never uses the name as an
// address: the device address comes from hipGetSymbolAddress, once per device
// with that device current, and only that pointer reaches the kernels.
static __device__ __align__(256) uint8_t scratch[ELSAR_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

elsar_status scratch_of_current_device(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return ELSAR_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return ELSAR_E_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return ELSAR_OK;
}
}  // namespace

extern "C" {

elsar_status elsar_sort_noalloc(const void* d_in, uint64_t n, void* d_out, const elsar_fit_params* p,
                                hipStream_t stream) {
  elsar_status s = check_params(p);
  if (s != ELSAR_OK) return s;
  if (n > ELSAR_MAX_DEVICE_RECORDS) return ELSAR_E_UNSUPPORTED;
  if (n == 0) return ELSAR_OK;
  if (!d_in || !d_out || !aligned16(d_in) || !aligned16(d_out)) return ELSAR_E_INVALID_ARG;
  const elsar_fit_params q = with_defaults(*p);
  if (sort_layout(q, resolve(q, n), n).bytes > (size_t)ELSAR_NOALLOC_SCRATCH_BYTES) return ELSAR_E_NO_MEMORY;
  void* ws = nullptr;
  s = scratch_of_current_device(&ws);
  if (s != ELSAR_OK) return s;
  return sort_job(d_in, n, d_out, q, ws, (size_t)ELSAR_NOALLOC_SCRATCH_BYTES, stream, false);
}

elsar_status elsar_sort_batch_workspace_size(const elsar_job* h_jobs, uint32_t njobs, const elsar_fit_params* p,
                                             size_t* bytes) {
  if (!bytes || (njobs && !h_jobs)) return ELSAR_E_INVALID_ARG;
  elsar_status s = check_params(p);
  if (s != ELSAR_OK) return s;
  if (p->key_bytes > kSortKeyBytes) return ELSAR_E_UNSUPPORTED;  // the small-job kernel sorts 12 key bytes
  if (p->key_len_offset) return ELSAR_E_UNSUPPORTED;             // fixed-length keys only
  BatchLayout bl;
  s = batch_layout(h_jobs, njobs, *p, &bl);
  if (s != ELSAR_OK) return s;
  *bytes = bl.bytes;
  return ELSAR_OK;
}

elsar_status elsar_sort_batch(const elsar_job* h_jobs, uint32_t njobs, const elsar_fit_params* p, void* d_ws,
                              size_t ws_bytes, hipStream_t stream) {
  if (njobs && !h_jobs) return ELSAR_E_INVALID_ARG;
  elsar_status s = check_params(p);
  if (s != ELSAR_OK) return s;
  if (p->key_bytes > kSortKeyBytes) return ELSAR_E_UNSUPPORTED;  // the small-job kernel sorts 12 key bytes
  if (p->key_len_offset) return ELSAR_E_UNSUPPORTED;             // fixed-length keys only
  if (njobs == 0) return ELSAR_OK;
  if (!d_ws || !aligned16(d_ws)) return ELSAR_E_INVALID_ARG;
  BatchLayout bl;
  s = batch_layout(h_jobs, njobs, *p, &bl);
  if (s != ELSAR_OK) return s;
  if (ws_bytes < bl.bytes) return ELSAR_E_NO_MEMORY;
  uint8_t* w = static_cast<uint8_t*>(d_ws);
  std::vector<uint8_t> key = plan_key(h_jobs, njobs, *p, d_ws, ws_bytes);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  auto it = std::find_if(g_plans.begin(), g_plans.end(), [&](const BatchPlan& x) { return x.key == key; });
  if (it == g_plans.end()) {
    BatchPlan plan;
    plan.key = std::move(key);
    plan.tiny = bl.tiny;
    plan.fit = fit_descriptors(h_jobs, *p, bl, w);
    plan.win = window_descriptors(h_jobs, *p, bl, w);
    s = build_plan(h_jobs, *p, bl, w, &plan);
    if (s != ELSAR_OK) return s;
    if (g_plans.size() >= kMaxPlans) {  // the oldest plan may still run: wait before freeing it
      HIP_TRY(hipDeviceSynchronize());
      BatchPlan& old = g_plans.back();
      (void)hipGraphExecDestroy(old.exec);
      (void)hipGraphDestroy(old.graph);
      g_plans.pop_back();
    }
    g_plans.push_front(std::move(plan));
    it = g_plans.begin();
  } else if (it != g_plans.begin()) {
    g_plans.splice(g_plans.begin(), g_plans, it);
    it = g_plans.begin();
  }
  // the small jobs' descriptors go to the workspace before every launch: the
  // caller may have used the workspace for something else in between
  if (!it->tiny.empty())
    HIP_TRY(hipMemcpyAsync(w + bl.tiny_desc, it->tiny.data(), it->tiny.size() * sizeof(TinyJob),
                           hipMemcpyHostToDevice, stream));
  if (!it->fit.empty())
    HIP_TRY(hipMemcpyAsync(w + bl.fit_desc, it->fit.data(), it->fit.size() * sizeof(FitJob),
                           hipMemcpyHostToDevice, stream));
  if (!it->win.empty())
    HIP_TRY(hipMemcpyAsync(w + bl.win_desc, it->win.data(), it->win.size() * sizeof(WinJob),
                           hipMemcpyHostToDevice, stream));
  HIP_TRY(hipGraphLaunch(it->exec, stream));
  return ELSAR_OK;
}

}  // extern "C"

namespace {

// ------------------------------------------------------------- host tier --
// The paper's larger-than-memory setting (Section 3) with host memory as the
// external store.  Two passes over the data, each record crossing the link
// four times in all:
//  * runs (Section 3.3's partitioning pass, written once): every chunk is
//    streamed to HBM, sorted there by the in-HBM method, and written back to
//    the fragment store as a sorted run; the global model's bucket counts of
//    the run are kept (its buckets are contiguous ranges of the sorted run);
//  * groups (Section 3.4): consecutive buckets whose records fit one pass are
//    read back, one slice per run, sorted in HBM and written to the output at
//    their offset (Section 3.5's concatenation at host level).
// A bucket alone larger than a pass whose keys are all equal is already in
// order across the runs (each run is stable, runs are in input order) and is
// copied through; one with different keys is refused.
constexpr uint64_t kDefaultChunkRecords = 40000000ull;  // 4 GB of 100-byte records
constexpr uint32_t kSampleBlocks = 4096;                  // strided blocks of the whole-input sample

// Partition buffer of one group pass: P records in exact regions for up to B
// buckets, no spill area.
PartLayout pass_layout(uint64_t P, uint32_t B, uint32_t R, uint32_t K) {
  PartLayout lay{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  lay.header = take(sizeof(PartHeader));
  lay.counts = take((size_t)B * 4);
  lay.cstride = counter_stride(B);
  lay.pcounts = lay.cstride > 1 ? take((size_t)B * lay.cstride * 4) : lay.counts;
  lay.caps = take((size_t)B * 4);
  lay.rstart = take((size_t)B * 4);
  lay.spill_off = take((size_t)B * 4);
  lay.mid_list = take((size_t)B * 4);
  lay.big_list = take((size_t)B * 4);
  lay.big2_list = take((size_t)B * 4);
  lay.psum = take((size_t)(B + kScanChunk - 1) / kScanChunk * sizeof(ScanPart));
  lay.spill_meta = take(0);
  lay.spill_map = take(0);
  lay.seg_leaf_cap = (uint32_t)std::min<uint64_t>(P / 32 + 4096, 0xFFFFFFFFull);
  lay.seg_leaf = take((size_t)lay.seg_leaf_cap * 16);
  lay.cap_slots = P;
  lay.total_slots = P;
  lay.slot_bytes = slot_bytes_for(R);
  size_t slot_area = (size_t)P * lay.slot_bytes;
  if (K > kSortKeyBytes) slot_area = std::max(slot_area, long_key_scratch_bytes(P, R));
  lay.slots = take(slot_area);
  lay.bytes = off;
  return lay;
}

// The big-bucket split stayed within its bounds: segments listed (seg_n[0])
// within the list's capacity, and no piece stack overflowed (seg_n[1]).
bool split_ok(const PartHeader& ph, const PartLayout& lay) {
  return ph.seg_n[1] == 0 && ph.seg_n[0] <= lay.seg_leaf_cap;
}

// Parameters of the in-HBM sort of one chunk (its own sample and model).
elsar_fit_params chunk_params(const elsar_fit_params& q) {
  elsar_fit_params c = q;
  c.num_buckets = 0;
  c.num_leaves = 0;
  c.sample_size = 0;
  return c;
}

struct HostLayout {
  Shape sh;                // the global model
  uint64_t C = 0, P = 0;   // chunk records, group-pass records
  size_t model = 0, fit = 0, counts = 0, ccount[2] = {0, 0}, offsets = 0, flag = 0;
  size_t region = 0;       // shared by the fit sample, the run pass and the group passes
  // run pass (offsets from region)
  size_t chunk[2] = {0, 0}, sorted[2] = {0, 0}, sort_ws = 0, sort_ws_bytes = 0;
  // group passes (offsets from region)
  size_t group = 0, part = 0, stage = 0;
  size_t bytes = 0;
  PartLayout lay;
};

HostLayout host_layout(const elsar_fit_params& q, uint64_t n, uint64_t C, uint64_t P) {
  HostLayout h;
  h.sh = resolve(q, n);
  h.C = std::max<uint64_t>(1, std::min<uint64_t>(C ? C : kDefaultChunkRecords, n));
  h.P = std::max<uint64_t>(1, P);
  const uint32_t R = q.record_bytes;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off += align_up(bytes);
    return o;
  };
  h.model = take(model_dev_bytes(h.sh, q.kind));
  h.fit = take(fit_ws_bytes(h.sh.S));
  h.counts = take((size_t)h.sh.B * 4);
  h.ccount[0] = take((size_t)h.sh.B * 4);
  h.ccount[1] = take((size_t)h.sh.B * 4);
  h.offsets = take(((size_t)h.sh.B + 1) * 8);
  h.flag = take(256);
  h.region = off;
  // the sample of the global model
  size_t r_fit = align_up((size_t)h.sh.S * R);
  // run pass: two input chunks, two sorted chunks, one chunk sort's workspace
  const elsar_fit_params cq = chunk_params(q);
  size_t r = 0;
  auto take_r = [&](size_t bytes) {
    size_t o = r;
    r += align_up(bytes);
    return o;
  };
  h.chunk[0] = take_r((size_t)h.C * R);
  h.chunk[1] = take_r((size_t)h.C * R);
  h.sorted[0] = take_r((size_t)h.C * R);
  h.sorted[1] = take_r((size_t)h.C * R);
  h.sort_ws_bytes = sort_layout(cq, resolve(cq, h.C), h.C).bytes;
  h.sort_ws = take_r(h.sort_ws_bytes);
  const size_t r_runs = r;
  // group passes: the gathered slices, the partition buffer, the output stage
  r = 0;
  h.group = take_r((size_t)h.P * R);
  h.lay = pass_layout(h.P, h.sh.B, R, q.key_bytes);
  h.part = take_r(h.lay.bytes);
  h.stage = take_r((size_t)h.P * R);
  const size_t r_groups = r;
  h.bytes = h.region + std::max(r_fit, std::max(r_runs, r_groups));
  return h;
}

// Largest group pass that fits ws_bytes (0 if not even one record does).
uint64_t pass_capacity(const elsar_fit_params& q, uint64_t n, uint64_t C, size_t ws_bytes) {
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    if (host_layout(q, n, C, mid).bytes <= ws_bytes) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct Streams {  // the upload stream and the events, released on every path (the stager copies back)
  hipStream_t h2d = nullptr;
  hipEvent_t loaded[2] = {}, freed[2] = {}, sorted[2] = {}, copied[2] = {}, counted[2] = {};
  ~Streams() {
    if (h2d) (void)hipStreamDestroy(h2d);
    for (auto* arr : {loaded, freed, sorted, copied, counted})
      for (int i = 0; i < 2; ++i)
        if (arr[i]) (void)hipEventDestroy(arr[i]);
  }
  bool init() {
    if (hipStreamCreateWithFlags(&h2d, hipStreamNonBlocking) != hipSuccess) return false;
    for (auto* arr : {loaded, freed, sorted, copied, counted})
      for (int i = 0; i < 2; ++i)
        if (hipEventCreateWithFlags(&arr[i], hipEventDisableTiming) != hipSuccess) return false;
    return true;
  }
};

// Copies between the device and host memory for the host tier.  Host memory
// that is not page-locked goes through pinned slots: the runtime's own path
// for it stages every copy on the calling thread (measured: 29.5 GB/s to the
// device, 17.7 GB/s back, the two directions barely overlapping).
//  * To the device (h2d, on the calling thread): a piece is copied into a
//    free slot by several CPU threads, then goes out by DMA on the given
//    stream while the next piece is copied.
//  * To the host (post_d2h, on a worker thread with a stream of its own): the
//    worker waits on the request's `after` event, moves the data piece by
//    piece into free slots by DMA, copies each landed piece to its
//    destination, and records the request's `done` event after its last
//    piece; page-locked destinations get one direct DMA.  The caller goes on
//    at once; wait_issued(id) returns when request id's done event has been
//    recorded (a stream may then wait on it), flush() when every request is
//    at its destination.
class Stager {
 public:
  static constexpr size_t kMaxSlotBytes = 128ull << 20;
  static constexpr int kInSlots = 4, kMaxOutSlots = 32;

  ~Stager() {
    if (worker_.joinable()) {
      (void)flush();
      {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
      }
      cv_.notify_all();
      worker_.join();
    }
    if (wst_) (void)hipStreamDestroy(wst_);
    for (Slot* arr : {in_, out_})
      for (int i = 0; i < (arr == in_ ? kInSlots : kMaxOutSlots); ++i) {
        if (arr[i].ev) (void)hipEventDestroy(arr[i].ev);
        if (arr[i].p) (void)hipHostFree(arr[i].p);
      }
  }

  // slots: whether any host buffer is pageable; bytes: the largest single
  // transfer to expect (a chunk).  Slots are at most 128 MB and about an
  // eighth of that transfer (at least 1 MB); enough out-slots for one such
  // transfer (4 to 32), four in-slots.  False: the worker or its stream could
  // not be started (nothing can be copied to the host then); without pinned
  // slots the pageable copies go the runtime's way, from the worker.
  bool init(bool slots, size_t bytes) {
    const unsigned hc = std::thread::hardware_concurrency();
    threads_ = hc ? std::min(8u, std::max(1u, hc / 2)) : 4u;
    if (hipStreamCreateWithFlags(&wst_, hipStreamNonBlocking) != hipSuccess) return false;
    slot_bytes_ = std::min(kMaxSlotBytes, std::max<size_t>(1u << 20, (bytes / 8 + 4095) & ~size_t(4095)));
    nout_ = (int)std::min<size_t>(kMaxOutSlots, std::max<size_t>(4, (bytes + slot_bytes_ - 1) / slot_bytes_));
    slots_ok_ = slots;
    for (Slot* arr : {in_, out_})
      for (int i = 0; slots && i < (arr == in_ ? kInSlots : nout_); ++i) {
        if (hipHostMalloc(reinterpret_cast<void**>(&arr[i].p), slot_bytes_, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&arr[i].ev, hipEventDisableTiming) != hipSuccess) {
          (void)hipGetLastError();
          slots_ok_ = false;
        }
      }
    for (int k = 0; k < nout_; ++k) free_.push_back(k);
    try {
      worker_ = std::thread([this] { work(); });
    } catch (...) {
      return false;
    }
    return true;
  }

  // whether p is page-locked host memory (then copied directly)
  static bool pinned(const void* p) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return a.type == hipMemoryTypeHost;
  }

  elsar_status h2d(void* dst, const void* src, size_t bytes, hipStream_t st, bool src_pinned) {
    if (src_pinned || !slots_ok_) {
      HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
      return ELSAR_OK;
    }
    for (size_t off = 0; off < bytes; off += slot_bytes_) {
      const size_t len = std::min(slot_bytes_, bytes - off);
      Slot& sl = in_[next_in_];
      next_in_ = (next_in_ + 1) % kInSlots;
      HIP_TRY(hipEventSynchronize(sl.ev));  // its previous DMA has read it
      copy(sl.p, static_cast<const uint8_t*>(src) + off, len);
      HIP_TRY(hipMemcpyAsync(static_cast<uint8_t*>(dst) + off, sl.p, len, hipMemcpyHostToDevice, st));
      HIP_TRY(hipEventRecord(sl.ev, st));
    }
    return ELSAR_OK;
  }

  // a device-to-host copy after `after` (may be null); `done` (may be null)
  // is recorded on the worker's stream after its last piece
  uint64_t post_d2h(void* dst, const void* src, size_t bytes, hipEvent_t after, hipEvent_t done, bool dst_pinned) {
    std::lock_guard<std::mutex> lk(mu_);
    Req r;
    r.dst = static_cast<uint8_t*>(dst);
    r.src = static_cast<const uint8_t*>(src);
    r.bytes = bytes;
    r.after = after;
    r.done = done;
    r.direct = dst_pinned || !slots_ok_;
    r.id = ++posted_;
    reqs_.push_back(r);
    cv_.notify_all();
    return r.id;
  }

  elsar_status wait_issued(uint64_t id) {
    std::unique_lock<std::mutex> lk(mu_);
    cv_.wait(lk, [&] { return issued_ >= id || failed_; });
    return failed_ ? ELSAR_E_HIP : ELSAR_OK;
  }

  elsar_status flush() {
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_.wait(lk, [&] { return (reqs_.empty() && inflight_.empty() && !draining_) || failed_; });
      if (failed_) return ELSAR_E_HIP;
    }
    HIP_TRY(hipStreamSynchronize(wst_));  // the direct copies
    return ELSAR_OK;
  }

 private:
  struct Slot {
    uint8_t* p = nullptr;
    hipEvent_t ev = nullptr;
    uint8_t* dst = nullptr;  // destination of the piece it holds
    size_t len = 0;
  };
  struct Req {
    uint8_t* dst = nullptr;
    const uint8_t* src = nullptr;
    size_t bytes = 0, issued = 0;
    hipEvent_t after = nullptr, done = nullptr;
    bool direct = false, waited = false;
    uint64_t id = 0;
  };

  // parallel memcpy on up to threads_ CPU threads (inline where a thread
  // cannot be started)
  void copy(void* dst, const void* src, size_t bytes) const {
    const unsigned T = bytes >= (16u << 20) ? threads_ : 1u;
    const size_t part = ((bytes + T - 1) / T + 4095) & ~size_t(4095);
    std::vector<std::thread> th;
    for (unsigned t = 1; t < T; ++t) {
      const size_t a = t * part;
      if (a >= bytes) break;
      const size_t len = std::min(part, bytes - a);
      uint8_t* d = static_cast<uint8_t*>(dst) + a;
      const uint8_t* s = static_cast<const uint8_t*>(src) + a;
      try {
        th.emplace_back([d, s, len] { std::memcpy(d, s, len); });
      } catch (...) {
        std::memcpy(d, s, len);
      }
    }
    std::memcpy(dst, src, std::min(part, bytes));
    for (auto& x : th) x.join();
  }

  // The worker: issue the front request's next piece while a slot is free,
  // else copy out the oldest piece in flight, else wait.
  void work() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      if (failed_) {  // drop everything; the callers see the failure
        reqs_.clear();
        inflight_.clear();
        cv_.notify_all();
        cv_.wait(lk, [&] { return stop_; });
        return;
      }
      if (!reqs_.empty() && (reqs_.front().direct || !free_.empty())) {
        Req& r = reqs_.front();  // only this thread pops the front
        bool ok = true;
        if (!r.waited) {
          r.waited = true;
          lk.unlock();
          if (r.after) ok = hipStreamWaitEvent(wst_, r.after, 0) == hipSuccess;
          lk.lock();
        }
        if (ok && r.direct) {
          lk.unlock();
          ok = hipMemcpyAsync(r.dst, r.src, r.bytes, hipMemcpyDeviceToHost, wst_) == hipSuccess;
          lk.lock();
          r.issued = r.bytes;
        } else if (ok) {
          const int k = free_.back();
          free_.pop_back();
          const size_t len = std::min(slot_bytes_, r.bytes - r.issued);
          Slot& sl = out_[k];
          sl.dst = r.dst + r.issued;
          sl.len = len;
          const uint8_t* src = r.src + r.issued;
          lk.unlock();
          ok = hipMemcpyAsync(sl.p, src, len, hipMemcpyDeviceToHost, wst_) == hipSuccess &&
               hipEventRecord(sl.ev, wst_) == hipSuccess;
          lk.lock();
          inflight_.push_back(k);
          r.issued += len;
        }
        if (ok && r.issued == r.bytes) {
          hipEvent_t done = r.done;
          const uint64_t id = r.id;
          lk.unlock();
          if (done) ok = hipEventRecord(done, wst_) == hipSuccess;
          lk.lock();
          reqs_.pop_front();
          issued_ = id;
          cv_.notify_all();
        }
        if (!ok) failed_ = true;
        continue;
      }
      if (!inflight_.empty()) {
        const int k = inflight_.front();
        inflight_.pop_front();
        draining_ = true;
        Slot& sl = out_[k];
        lk.unlock();
        const bool ok = hipEventSynchronize(sl.ev) == hipSuccess;
        if (ok) copy(sl.dst, sl.p, sl.len);
        lk.lock();
        draining_ = false;
        free_.push_back(k);
        if (!ok) failed_ = true;
        cv_.notify_all();
        continue;
      }
      if (stop_) return;
      cv_.wait(lk, [&] {
        return stop_ || !inflight_.empty() || (!reqs_.empty() && (reqs_.front().direct || !free_.empty()));
      });
    }
  }

  Slot in_[kInSlots], out_[kMaxOutSlots];
  int next_in_ = 0, nout_ = 4;
  size_t slot_bytes_ = kMaxSlotBytes;
  unsigned threads_ = 4;
  bool slots_ok_ = false;
  hipStream_t wst_ = nullptr;
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<Req> reqs_;     // requests not fully issued, in order
  std::deque<int> inflight_;  // out slots holding a piece, oldest first
  std::vector<int> free_;     // out slots free
  uint64_t posted_ = 0, issued_ = 0;
  bool draining_ = false, stop_ = false, failed_ = false;
  std::thread worker_;
};

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// The whole-input sample for the global model: nb evenly spaced blocks of bs
// consecutive records (systematic sampling with one random start), gathered
// by one strided copy.  Returns the records copied.
elsar_status gather_sample(const uint8_t* in, uint64_t n, uint32_t R, uint64_t S, uint64_t seed, uint8_t* dst,
                           hipStream_t st, uint64_t* got) {
  const uint64_t nb = std::min<uint64_t>(S, kSampleBlocks);
  const uint64_t bs = S / nb, pitch = n / nb;  // bs <= pitch since S <= n
  // a start in [0, pitch - bs] from the seed (SplitMix64 output function)
  uint64_t z = seed + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const uint64_t start = (pitch > bs) ? z % (pitch - bs + 1) : 0;
  HIP_TRY(hipMemcpy2DAsync(dst, bs * R, in + start * R, pitch * R, bs * R, nb, hipMemcpyHostToDevice, st));
  *got = nb * bs;
  return ELSAR_OK;
}

}  // namespace

extern "C" {

elsar_status elsar_sort_host_workspace_size(const elsar_fit_params* p, uint64_t n, uint64_t chunk_records,
                                            uint64_t pass_records, size_t* bytes) {
  if (!bytes) return ELSAR_E_INVALID_ARG;
  elsar_status s = check_params(p);
  if (s != ELSAR_OK) return s;
  if (n > 0xFFFFFFFFull) return ELSAR_E_UNSUPPORTED;
  const elsar_fit_params q = with_defaults(*p);
  *bytes = host_layout(q, std::max<uint64_t>(n, 1), chunk_records, pass_records ? pass_records : n).bytes;
  return ELSAR_OK;
}

elsar_status elsar_sort_host(const void* h_in, uint64_t n, void* h_out, void* h_frag, const elsar_fit_params* p,
                             uint64_t chunk_records, uint64_t pass_records, uint32_t flags, void* d_ws,
                             size_t ws_bytes, hipStream_t stream, elsar_host_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  elsar_status s = check_params(p);
  if (s != ELSAR_OK) return s;
  if (n > 0xFFFFFFFFull) return ELSAR_E_UNSUPPORTED;  // chunk and group positions are 32-bit
  if (flags & ~(uint32_t)ELSAR_HOST_SAMPLE_FIRST_CHUNK) return ELSAR_E_INVALID_ARG;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  if (n == 0) return ELSAR_OK;
  if (!h_in || !h_out || !h_frag || !d_ws || !aligned16(d_ws) || !aligned16(h_in) || !aligned16(h_out) ||
      !aligned16(h_frag))
    return ELSAR_E_INVALID_ARG;
  const elsar_fit_params q = with_defaults(*p);
  const uint32_t R = q.record_bytes;
  const uint8_t* in = static_cast<const uint8_t*>(h_in);
  uint8_t* out = static_cast<uint8_t*>(h_out);
  uint8_t* frag = static_cast<uint8_t*>(h_frag);
  auto overlap = [&](const uint8_t* a, const uint8_t* b) { return a < b + n * R && b < a + n * R; };
  if (overlap(in, out) || overlap(frag, out)) return ELSAR_E_INVALID_ARG;
  if (frag != in && overlap(frag, in)) return ELSAR_E_INVALID_ARG;
  uint64_t P = pass_capacity(q, n, chunk_records, ws_bytes);
  if (P == 0) return ELSAR_E_NO_MEMORY;
  if (pass_records) P = std::min(P, pass_records);
  const HostLayout hl = host_layout(q, n, chunk_records, P);
  uint8_t* w = static_cast<uint8_t*>(d_ws);
  uint8_t* region = w + hl.region;
  Streams ss;
  if (!ss.init()) return ELSAR_E_HIP;
  uint64_t link = 0;
  // buffers that are not page-locked go through the stager's pinned slots
  const bool in_pinned = Stager::pinned(in), out_pinned = Stager::pinned(out), frag_pinned = Stager::pinned(frag);
  Stager stg;
  if (!stg.init(!(in_pinned && out_pinned && frag_pinned), (size_t)std::min<uint64_t>(hl.C, n) * R)) return ELSAR_E_HIP;

  // 1. the global model: on a sample spread over the whole input, or (flag) on
  //    the first chunk only, as the paper samples the first batch that one
  //    reader reads (Section 3.1)
  elsar_model m{};
  m.p = q;
  m.B = hl.sh.B;
  m.L = hl.sh.L;
  m.Lm = hl.sh.Lm;
  place_model(&m, w + hl.model);
  {
    uint64_t ns = 0;
    if (flags & ELSAR_HOST_SAMPLE_FIRST_CHUNK) {
      ns = std::min<uint64_t>(hl.C, n);
      HIP_TRY(hipMemcpyAsync(region, in, ns * R, hipMemcpyHostToDevice, stream));
    } else {
      s = gather_sample(in, n, R, hl.sh.S, q.seed, region, stream, &ns);
      if (s != ELSAR_OK) return s;
    }
    link += ns * R;
    m.S = std::min<uint64_t>(hl.sh.S, ns);
    s = do_fit(&m, region, ns, w + hl.fit, fit_ws_bytes(hl.sh.S), stream);
    if (s != ELSAR_OK) return s;
  }
  HIP_TRY(hipStreamSynchronize(stream));
  const double t_fit = ms_since(t0);
  const MlpState* ms = m.has_mlp ? &m.ms : nullptr;

  // 2. runs: each chunk sorted in HBM and written to the fragment store at its
  //    own place; its counts per global bucket kept for the group passes
  const uint64_t nchunks = (n + hl.C - 1) / hl.C;
  // the runs' counts land in page-locked memory: a copy to pageable memory
  // would block this thread until the copy stream reached it
  struct PinnedCounts {
    uint32_t* p = nullptr;
    ~PinnedCounts() {
      if (p) (void)hipHostFree(p);
    }
  } pc;
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&pc.p), (size_t)nchunks * m.B * 4, hipHostMallocDefault));
  const elsar_fit_params cq = chunk_params(q);
  uint64_t run_req[2] = {0, 0};  // the copy request of the last run in each buffer
  for (uint64_t c = 0; c < nchunks; ++c) {
    const int k = (int)(c & 1u);
    const uint64_t first = c * hl.C, cnt = std::min<uint64_t>(hl.C, n - first);
    uint8_t* buf = region + hl.chunk[k];
    uint8_t* srt = region + hl.sorted[k];
    uint32_t* cc = reinterpret_cast<uint32_t*>(w + hl.ccount[k]);
    if (c >= 2) HIP_TRY(hipStreamWaitEvent(ss.h2d, ss.freed[k], 0));
    s = stg.h2d(buf, in + first * R, cnt * R, ss.h2d, in_pinned);
    if (s != ELSAR_OK) return s;
    HIP_TRY(hipEventRecord(ss.loaded[k], ss.h2d));
    HIP_TRY(hipStreamWaitEvent(stream, ss.loaded[k], 0));
    if (c >= 2) {  // sorted[k] and cc[k] are out: the copies of run c - 2 are done
      s = stg.wait_issued(run_req[k]);
      if (s != ELSAR_OK) return s;
      HIP_TRY(hipStreamWaitEvent(stream, ss.copied[k], 0));
    }
    s = sort_job(buf, cnt, srt, cq, region + hl.sort_ws, hl.sort_ws_bytes, stream, false);
    if (s != ELSAR_OK) return s;
    HIP_TRY(hipEventRecord(ss.freed[k], stream));
    HIP_TRY(launch_fill_u32(cc, m.B, 0u, stream));
    HIP_TRY(launch_count(m.hdr, m.leaves, ms, srt, cnt, R, cc, stream, vkey(q)));
    HIP_TRY(hipEventRecord(ss.sorted[k], stream));
    (void)stg.post_d2h(pc.p + (size_t)c * m.B, cc, (size_t)m.B * 4, ss.sorted[k], nullptr, true);
    run_req[k] = stg.post_d2h(frag + first * R, srt, cnt * R, nullptr, ss.copied[k], frag_pinned);
    link += 2 * cnt * R;
  }
  HIP_TRY(hipStreamSynchronize(stream));
  s = stg.flush();  // the runs are in the fragment store before any group reads them
  if (s != ELSAR_OK) return s;
  const double t_runs = ms_since(t0);

  // 3. group passes over consecutive buckets whose records fit one pass
  auto ccounts = [&](uint64_t c, uint32_t b) { return pc.p[(size_t)c * m.B + b]; };
  std::vector<uint64_t> counts(m.B, 0);
  for (uint64_t c = 0; c < nchunks; ++c)
    for (uint32_t b = 0; b < m.B; ++b) counts[b] += ccounts(c, b);
  // run c's bucket b starts at pre[c][b] in the run (exclusive sums)
  std::vector<std::vector<uint32_t>> pre(nchunks, std::vector<uint32_t>(m.B + 1));
  for (uint64_t c = 0; c < nchunks; ++c) {
    uint32_t acc = 0;
    for (uint32_t b = 0; b < m.B; ++b) {
      pre[c][b] = acc;
      acc += ccounts(c, b);
    }
    pre[c][m.B] = acc;
    if (acc != std::min<uint64_t>(hl.C, n - c * hl.C)) return ELSAR_E_HIP;  // counts must cover the run
  }
  struct Group {
    uint32_t lo, hi;  // buckets lo .. hi-1
    uint64_t first, total;
    bool copy;        // one bucket above a pass: all keys equal, copied through in run order
  };
  std::vector<Group> groups;
  uint64_t done = 0;
  for (uint32_t b = 0; b < m.B;) {
    Group g{b, b, done, 0, false};
    while (g.hi < m.B && g.total + counts[g.hi] <= hl.P) g.total += counts[g.hi++];
    if (g.hi == g.lo) {
      g.hi = b + 1;
      g.total = counts[b];
      g.copy = true;
    }
    groups.push_back(g);
    done += g.total;
    b = g.hi;
  }
  if (done != n) return ELSAR_E_HIP;  // the counts must cover every record
  uint32_t* counts_dev = reinterpret_cast<uint32_t*>(w + hl.counts);
  {
    std::vector<uint32_t> c32(m.B);
    for (uint32_t b = 0; b < m.B; ++b) c32[b] = (uint32_t)counts[b];
    HIP_TRY(hipMemcpyAsync(counts_dev, c32.data(), (size_t)m.B * 4, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
  }
  uint8_t* gbuf = region + hl.group;
  uint8_t* part = region + hl.part;
  uint8_t* stage = region + hl.stage;
  uint64_t* offsets = reinterpret_cast<uint64_t*>(w + hl.offsets);
  uint32_t* flag = reinterpret_cast<uint32_t*>(w + hl.flag);
  HIP_TRY(launch_fill_u32(flag, 1, 0u, stream));
  bool stage_busy = false, gbuf_busy = false;
  uint64_t out_req = 0;  // the copy request of the stage's last output
  bool sorted_once = false;  // the pass buffer's split bookkeeping is valid once a group was sorted
  uint32_t copy_groups = 0;
  // bytes compared by the copy pass: the key, and with variable-length keys
  // every byte up to the length byte (equal bytes there mean equal keys)
  const uint32_t cmp_bytes = q.key_len_offset ? q.key_len_offset + 1 : q.key_bytes;
  for (const Group& g : groups) {
    if (g.total == 0) continue;
    if (g.copy) {
      // a bucket above a pass: its slices in run order, piece by piece through
      // the stage; a kernel checks that every key equals the bucket's first
      ++copy_groups;
      uint64_t put = 0;
      bool have_ref = false;
      uint64_t c = 0, pos = pre[0][g.lo];
      while (put < g.total) {
        if (stage_busy) {
          s = stg.wait_issued(out_req);
          if (s != ELSAR_OK) return s;
          HIP_TRY(hipStreamWaitEvent(ss.h2d, ss.copied[0], 0));
        }
        uint64_t got = 0;
        while (got < hl.P && c < nchunks) {
          const uint64_t end = pre[c][g.hi];
          const uint64_t take = std::min<uint64_t>(end - pos, hl.P - got);
          if (take) {
            s = stg.h2d(stage + got * R, frag + (c * hl.C + pos) * R, take * R, ss.h2d, frag_pinned);
            if (s != ELSAR_OK) return s;
          }
          got += take;
          pos += take;
          if (pos == end && ++c < nchunks) pos = pre[c][g.lo];
        }
        HIP_TRY(hipEventRecord(ss.loaded[0], ss.h2d));
        HIP_TRY(hipStreamWaitEvent(stream, ss.loaded[0], 0));
        if (!have_ref) {
          HIP_TRY(hipMemcpyAsync(flag + 32, stage, cmp_bytes, hipMemcpyDeviceToDevice, stream));
          have_ref = true;
        }
        HIP_TRY(launch_keys_differ(stage, got, R, cmp_bytes, reinterpret_cast<const uint8_t*>(flag + 32), flag,
                                   stream));
        HIP_TRY(hipEventRecord(ss.sorted[0], stream));
        out_req = stg.post_d2h(out + (g.first + put) * R, stage, got * R, ss.sorted[0], ss.copied[0], out_pinned);
        stage_busy = true;
        put += got;
        link += 2 * got * R;
      }
      continue;
    }
    // gather the group's slice of every run into gbuf (after the previous
    // group's partition has read it)
    if (gbuf_busy) HIP_TRY(hipStreamWaitEvent(ss.h2d, ss.freed[0], 0));
    uint64_t got = 0;
    for (uint64_t c = 0; c < nchunks; ++c) {
      const uint64_t a = pre[c][g.lo], e = pre[c][g.hi];
      if (e > a) {
        s = stg.h2d(gbuf + got * R, frag + (c * hl.C + a) * R, (e - a) * R, ss.h2d, frag_pinned);
        if (s != ELSAR_OK) return s;
      }
      got += e - a;
    }
    if (got != g.total) return ELSAR_E_HIP;
    link += 2 * got * R;
    HIP_TRY(hipEventRecord(ss.loaded[0], ss.h2d));
    HIP_TRY(hipStreamWaitEvent(stream, ss.loaded[0], 0));
    const uint32_t nb = g.hi - g.lo;
    HIP_TRY(launch_exact_regions(counts_dev, g.lo, nb, g.total, part, hl.lay, stream));
    PassFilter f{0, g.lo, g.hi};  // every record of gbuf is in the group; its position breaks ties
    HIP_TRY(launch_partition(m.hdr, m.leaves, ms, gbuf, g.total, R, vkey(q), part, hl.lay, stream, &f));
    HIP_TRY(hipEventRecord(ss.freed[0], stream));
    gbuf_busy = true;
    // the regions are exact: a record that found its region full would mean
    // the run counts and the placement disagree; stop before a sort reads it.
    // The header still holds the previous group's split bookkeeping (the
    // bucket sorts clear it), checked here too.
    {
      PartHeader ph;
      HIP_TRY(hipMemcpyAsync(&ph, part + hl.lay.header, sizeof(ph), hipMemcpyDeviceToHost, stream));
      HIP_TRY(hipStreamSynchronize(stream));
      if (ph.spill_count != 0 || (sorted_once && !split_ok(ph, hl.lay))) return ELSAR_E_HIP;
    }
    HIP_TRY(launch_scan_counts(part, hl.lay, nb, offsets, stream));
    if (stage_busy) {  // the previous output is out
      s = stg.wait_issued(out_req);
      if (s != ELSAR_OK) return s;
      HIP_TRY(hipStreamWaitEvent(stream, ss.copied[0], 0));
    }
    HIP_TRY(launch_bucket_sort_small(part, hl.lay, nb, offsets, R, sort_bytes(q), stage, stream, vkey(q)));
    HIP_TRY(launch_bucket_sort_large(part, hl.lay, nb, g.total, offsets, R, sort_bytes(q), stage, stream,
                                     vkey(q)));
    HIP_TRY(launch_long_key_fixup(stage, g.total, R, q.key_bytes, part + hl.lay.slots, stream));
    sorted_once = true;
    HIP_TRY(hipEventRecord(ss.sorted[0], stream));
    out_req = stg.post_d2h(out + g.first * R, stage, g.total * R, ss.sorted[0], ss.copied[0], out_pinned);
    stage_busy = true;
  }
  HIP_TRY(hipStreamSynchronize(ss.h2d));
  HIP_TRY(hipStreamSynchronize(stream));
  s = stg.flush();  // every group's records are in the output
  if (s != ELSAR_OK) return s;
  // every bucket copied through held one key only; the last group's split
  // stayed within its bounds
  uint32_t bad = 0;
  HIP_TRY(hipMemcpy(&bad, flag, 4, hipMemcpyDeviceToHost));
  if (bad) return ELSAR_E_UNSUPPORTED;  // a bucket above a pass whose keys differ
  if (sorted_once) {
    PartHeader ph;
    HIP_TRY(hipMemcpy(&ph, part + hl.lay.header, sizeof(ph), hipMemcpyDeviceToHost));
    if (!split_ok(ph, hl.lay)) return ELSAR_E_HIP;
  }
  if (stats) {
    stats->chunk_records = hl.C;
    stats->pass_records = hl.P;
    stats->passes = (uint32_t)groups.size();
    stats->num_buckets = m.B;
    stats->runs = (uint32_t)nchunks;
    stats->copy_passes = copy_groups;
    stats->link_bytes = link;
    stats->fit_ms = (float)t_fit;
    stats->count_ms = (float)(t_runs - t_fit);
    stats->total_ms = (float)ms_since(t0);
    stats->passes_ms = stats->total_ms - (float)t_runs;
  }
  return ELSAR_OK;
}

}  // extern "C"

namespace {
void fill_model_info(const elsar_model* m, const ModelHeader& h, uint64_t n_fit, elsar_model_info* info) {
  std::memset(info, 0, sizeof(*info));
  info->kind_used = h.kind_used == 2 ? (uint32_t)ELSAR_MODEL_SPLINE : h.kind_used;  // header: 2 = spline root
  info->mlp_rejected = h.mlp_rejected;
  info->num_buckets = m->B;
  info->num_leaves = (m->has_mlp && h.kind_used != 0) ? m->Lm : m->L;
  const bool eq = m->has_mlp && !h.mlp_skip;  // the equi-depth leaves were fitted
  info->mlp_leaves = eq ? m->Lm : 0;
  info->spline_segments = eq ? spline_segments(m->Lm) : 0;
  info->sample_size = m->S;
  info->n_fit = n_fit;
  info->root_a0 = h.a0;
  info->root_a1 = h.a1;
  info->max_sample_bucket = h.max_sample_bucket;
  info->opt_sample_bucket = h.opt_sample_bucket;
  info->rmi_max_sample_bucket = h.max_rmi;
  info->eq_max_sample_bucket = h.max_eq;
  info->net_max_sample_bucket = h.max_net;
  info->rmi_gate_passed = h.rmi_ok;
  info->perfect_sample_bucket = h.perfect;
}
}  // namespace

extern "C" {

elsar_status elsar_model_info_get(const elsar_model* m, elsar_model_info* info) {
  if (!m || !info) return ELSAR_E_INVALID_ARG;
  ModelHeader h;
  HIP_TRY(hipMemcpy(&h, m->hdr, sizeof(h), hipMemcpyDeviceToHost));
  fill_model_info(m, h, m->n, info);
  return ELSAR_OK;
}

elsar_status elsar_sort_batch_model_info(const elsar_job* h_jobs, uint32_t njobs, const elsar_fit_params* p,
                                         const void* d_ws, size_t ws_bytes, uint32_t job, elsar_model_info* info) {
  if (!h_jobs || !info || !d_ws || job >= njobs) return ELSAR_E_INVALID_ARG;
  elsar_status s = check_params(p);
  if (s != ELSAR_OK) return s;
  if (h_jobs[job].n <= kSmallCap) return ELSAR_E_INVALID_ARG;
  BatchLayout bl;
  s = batch_layout(h_jobs, njobs, *p, &bl);
  if (s != ELSAR_OK) return s;
  if (ws_bytes < bl.bytes) return ELSAR_E_NO_MEMORY;
  const elsar_model m = job_model(h_jobs, *p, bl, static_cast<uint8_t*>(const_cast<void*>(d_ws)), job);
  ModelHeader h;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(&h, m.hdr, sizeof(h), hipMemcpyDeviceToHost));
  fill_model_info(&m, h, h.n_fit, info);
  return ELSAR_OK;
}

elsar_status elsar_model_leaves(const elsar_model* m, uint64_t* h_base, float* h_slope, float* h_icpt,
                                uint32_t* h_lo, uint32_t* h_hi) {
  if (!m) return ELSAR_E_INVALID_ARG;
  ModelHeader h;
  HIP_TRY(hipMemcpy(&h, m->hdr, sizeof(h), hipMemcpyDeviceToHost));
  const bool mlp = m->has_mlp && h.kind_used != 0;
  const Leaf* src = mlp ? m->ms.leaves : m->leaves;
  std::vector<Leaf> lv(mlp ? m->Lm : m->L);
  HIP_TRY(hipMemcpy(lv.data(), src, lv.size() * sizeof(Leaf), hipMemcpyDeviceToHost));
  for (uint32_t j = 0; j < lv.size(); ++j) {
    if (h_base) h_base[j] = lv[j].base;
    if (h_slope) h_slope[j] = lv[j].c;
    if (h_icpt) h_icpt[j] = lv[j].b;
    if (h_lo) h_lo[j] = lv[j].lo;
    if (h_hi) h_hi[j] = lv[j].hi;
  }
  return ELSAR_OK;
}

elsar_status elsar_model_spline_get(const elsar_model* m, uint64_t* h_knots, uint64_t* h_bound, uint32_t* h_first) {
  if (!m || !m->has_mlp) return ELSAR_E_INVALID_ARG;
  ModelHeader h;
  HIP_TRY(hipMemcpy(&h, m->hdr, sizeof(h), hipMemcpyDeviceToHost));
  if (h.mlp_skip) return ELSAR_E_INVALID_ARG;  // automatic choice kept the linear root: nothing fitted
  const size_t K = spline_segments(m->Lm);
  if (h_knots) HIP_TRY(hipMemcpy(h_knots, m->ms.knots, (K + 1) * 8, hipMemcpyDeviceToHost));
  if (h_bound) HIP_TRY(hipMemcpy(h_bound, m->ms.bound, ((size_t)m->Lm + 1) * 8, hipMemcpyDeviceToHost));
  if (h_first) HIP_TRY(hipMemcpy(h_first, m->ms.first, ((size_t)m->Lm + 1) * 4, hipMemcpyDeviceToHost));
  return ELSAR_OK;
}

elsar_status elsar_model_mlp_get(const elsar_model* m, float* h_params, uint64_t* h_knots, uint64_t* h_bound,
                                 uint32_t* h_first) {
  if (!m || !m->has_mlp || m->p.kind != ELSAR_MODEL_MLP) return ELSAR_E_INVALID_ARG;
  if (h_params) HIP_TRY(hipMemcpy(h_params, m->ms.master, (size_t)kMlpParams * 4, hipMemcpyDeviceToHost));
  if (h_knots) HIP_TRY(hipMemcpy(h_knots, m->ms.M->h.q, 9 * 8, hipMemcpyDeviceToHost));
  if (h_bound) HIP_TRY(hipMemcpy(h_bound, m->ms.bound, ((size_t)m->Lm + 1) * 8, hipMemcpyDeviceToHost));
  if (h_first) HIP_TRY(hipMemcpy(h_first, m->ms.first, ((size_t)m->Lm + 1) * 4, hipMemcpyDeviceToHost));
  return ELSAR_OK;
}

namespace {
// Device scratch of the verification entry points, freed on every path.
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

elsar_status mlp_block_from_host(const float* h_params, const uint64_t* h_knots, DevBuf& buf, size_t extra,
                                 MlpBlock** M, uint8_t** rest) {
  const size_t head = align_up(sizeof(MlpBlock)) + align_up((size_t)kMlpParams * 4) + align_up(9 * 8);
  if (hipMalloc(&buf.p, head + extra) != hipSuccess) return ELSAR_E_NO_MEMORY;
  uint8_t* b = static_cast<uint8_t*>(buf.p);
  *M = reinterpret_cast<MlpBlock*>(b);
  float* d_params = reinterpret_cast<float*>(b + align_up(sizeof(MlpBlock)));
  uint64_t* d_q = reinterpret_cast<uint64_t*>(b + align_up(sizeof(MlpBlock)) + align_up((size_t)kMlpParams * 4));
  *rest = b + head;
  HIP_TRY(hipMemcpy(d_params, h_params, (size_t)kMlpParams * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d_q, h_knots, 9 * 8, hipMemcpyHostToDevice));
  HIP_TRY(launch_mlp_params_to_block(d_params, d_q, *M, nullptr));
  return ELSAR_OK;
}
}  // namespace

elsar_status elsar_mlp_forward(const float* h_params, const uint64_t* h_knots, const uint64_t* h_codes, uint64_t n,
                               float* h_y) {
  if (!h_params || !h_knots || (n && (!h_codes || !h_y))) return ELSAR_E_INVALID_ARG;
  if (n > (1ull << 32)) return ELSAR_E_UNSUPPORTED;
  if (n == 0) return ELSAR_OK;
  DevBuf buf;
  MlpBlock* M = nullptr;
  uint8_t* rest = nullptr;
  elsar_status s = mlp_block_from_host(h_params, h_knots, buf, align_up(n * 8) + align_up(n * 4), &M, &rest);
  if (s != ELSAR_OK) return s;
  uint64_t* d_codes = reinterpret_cast<uint64_t*>(rest);
  float* d_y = reinterpret_cast<float*>(rest + align_up(n * 8));
  HIP_TRY(hipMemcpy(d_codes, h_codes, n * 8, hipMemcpyHostToDevice));
  HIP_TRY(launch_mlp_eval(M, d_codes, n, d_y, nullptr));
  HIP_TRY(hipMemcpy(h_y, d_y, n * 4, hipMemcpyDeviceToHost));
  return ELSAR_OK;
}

elsar_status elsar_mlp_gradient(const float* h_params, const uint64_t* h_knots, const uint64_t* h_codes,
                                const float* h_targets, float* h_grad, float* h_loss) {
  if (!h_params || !h_knots || !h_codes || !h_targets || !h_grad) return ELSAR_E_INVALID_ARG;
  const size_t rows = kMlpGradRows;
  DevBuf buf;
  MlpBlock* M = nullptr;
  uint8_t* rest = nullptr;
  elsar_status s = mlp_block_from_host(h_params, h_knots, buf,
                                       align_up(rows * 8) + align_up(rows * 4) + align_up((size_t)kMlpParams * 4) + 256,
                                       &M, &rest);
  if (s != ELSAR_OK) return s;
  uint64_t* d_codes = reinterpret_cast<uint64_t*>(rest);
  float* d_t = reinterpret_cast<float*>(rest + align_up(rows * 8));
  float* d_g = reinterpret_cast<float*>(rest + align_up(rows * 8) + align_up(rows * 4));
  float* d_loss = reinterpret_cast<float*>(rest + align_up(rows * 8) + align_up(rows * 4) +
                                           align_up((size_t)kMlpParams * 4));
  HIP_TRY(hipMemcpy(d_codes, h_codes, rows * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d_t, h_targets, rows * 4, hipMemcpyHostToDevice));
  HIP_TRY(launch_mlp_grad(M, d_codes, d_t, d_g, d_loss, nullptr));
  HIP_TRY(hipMemcpy(h_grad, d_g, (size_t)kMlpParams * 4, hipMemcpyDeviceToHost));
  if (h_loss) HIP_TRY(hipMemcpy(h_loss, d_loss, 4, hipMemcpyDeviceToHost));
  return ELSAR_OK;
}

elsar_status elsar_mlp_train_step(const float* h_params, const float* h_adam, const uint64_t* h_knots,
                                  const uint64_t* h_codes, const float* h_targets, uint32_t step, float lr,
                                  float* h_params_out, float* h_adam_out, float* h_grad, float* h_loss) {
  if (!h_params || !h_adam || !h_knots || !h_codes || !h_targets || !h_params_out || !h_adam_out)
    return ELSAR_E_INVALID_ARG;
  if (step == 0 || !(lr >= 0.0f)) return ELSAR_E_INVALID_ARG;
  const size_t rows = kMlpGradRows, P = kMlpParams;
  DevBuf buf;
  MlpBlock* M = nullptr;
  uint8_t* rest = nullptr;
  elsar_status s = mlp_block_from_host(h_params, h_knots, buf,
                                       align_up(rows * 8) + align_up(rows * 4) + align_up(P * 4) + align_up(P * 8) +
                                           align_up(P * 4) + 256,
                                       &M, &rest);
  if (s != ELSAR_OK) return s;
  uint64_t* d_codes = reinterpret_cast<uint64_t*>(rest);
  rest += align_up(rows * 8);
  float* d_t = reinterpret_cast<float*>(rest);
  rest += align_up(rows * 4);
  float* d_p = reinterpret_cast<float*>(rest);
  rest += align_up(P * 4);
  float* d_a = reinterpret_cast<float*>(rest);
  rest += align_up(P * 8);
  float* d_g = reinterpret_cast<float*>(rest);
  rest += align_up(P * 4);
  float* d_loss = reinterpret_cast<float*>(rest);
  HIP_TRY(hipMemcpy(d_codes, h_codes, rows * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d_t, h_targets, rows * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d_p, h_params, P * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(d_a, h_adam, P * 8, hipMemcpyHostToDevice));
  HIP_TRY(launch_mlp_step(M, d_p, d_a, d_codes, d_t, step, lr, d_g, d_loss, nullptr));
  HIP_TRY(hipMemcpy(h_params_out, d_p, P * 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(h_adam_out, d_a, P * 8, hipMemcpyDeviceToHost));
  if (h_grad) HIP_TRY(hipMemcpy(h_grad, d_g, P * 4, hipMemcpyDeviceToHost));
  if (h_loss) HIP_TRY(hipMemcpy(h_loss, d_loss, 4, hipMemcpyDeviceToHost));
  return ELSAR_OK;
}

elsar_status elsar_partition_stats_get(const elsar_model* m, const void* d_part, size_t part_bytes,
                                       elsar_partition_stats* st) {
  if (!m || !d_part || !st) return ELSAR_E_INVALID_ARG;
  if (part_bytes < sizeof(PartHeader)) return ELSAR_E_NO_MEMORY;
  PartHeader h;
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(&h, d_part, sizeof(h), hipMemcpyDeviceToHost));
  std::memset(st, 0, sizeof(*st));
  st->n = h.n;
  st->num_buckets = h.B;
  st->spill_count = h.spill_count;
  st->mid_buckets = h.n_mid + h.n_mid_hi;
  st->big_buckets = h.n_big;
  st->max_bucket = h.max_count;
  st->mid_records = h.mid_records;
  st->big_records = h.big_records;
  st->split_segments = h.seg_n[0];
  st->split_segment_cap =
      part_layout(h.n, m->B, m->p.record_bytes, m->p.region_pct, m->p.key_bytes).seg_leaf_cap;
  st->split_overflow = h.seg_n[1];
  return ELSAR_OK;
}

elsar_status elsar_set_timing(int enabled) {
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (enabled && g_timing.ev.empty()) {
    g_timing.ev.resize((size_t)kTimingSlots * kTimedPhases);
    g_timing.have.assign(kTimingSlots, 0);
    for (auto& e : g_timing.ev)
      if (hipEventCreate(&e) != hipSuccess) return ELSAR_E_HIP;
  }
  g_timing.on = enabled != 0;
  g_timing.next = 0;
  g_timing.used = 0;
  return ELSAR_OK;
}

elsar_status elsar_timings_get(elsar_timings* t) {
  if (!t) return ELSAR_E_INVALID_ARG;
  std::memset(t, 0, sizeof(*t));
  std::lock_guard<std::mutex> lk(g_timing.mu);
  if (g_timing.ev.empty() || g_timing.used == 0) return ELSAR_OK;
  double acc[kTimedPhases - 1] = {}, tot = 0;
  int cnt[kTimedPhases - 1] = {}, ctot = 0;
  for (int s = 0; s < g_timing.used; ++s) {
    hipEvent_t* e = &g_timing.ev[(size_t)s * kTimedPhases];
    uint8_t hv = g_timing.have[s];
    for (int i = 0; i < kTimedPhases; ++i)
      if ((hv >> i) & 1u) HIP_TRY(hipEventSynchronize(e[i]));
    for (int i = 0; i + 1 < kTimedPhases; ++i) {
      if (((hv >> i) & 1u) && ((hv >> (i + 1)) & 1u)) {
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e[i], e[i + 1]));
        acc[i] += ms;
        cnt[i]++;
      }
    }
    int first = -1, last = -1;
    for (int i = 0; i < kTimedPhases; ++i)
      if ((hv >> i) & 1u) {
        if (first < 0) first = i;
        last = i;
      }
    if (first >= 0 && last > first) {
      float ms = 0;
      HIP_TRY(hipEventElapsedTime(&ms, e[first], e[last]));
      tot += ms;
      ctot++;
    }
  }
  auto mean = [&](int i) { return cnt[i] ? (float)(acc[i] / cnt[i]) : 0.0f; };
  t->sample_fit_ms = mean(0);
  t->partition_ms = mean(1);
  t->scan_ms = mean(2);
  t->bucket_sort_lds_ms = mean(3);
  t->bucket_sort_rest_ms = mean(4);
  t->total_ms = ctot ? (float)(tot / ctot) : 0.0f;
  t->calls = (uint32_t)g_timing.used;
  return ELSAR_OK;
}

const char* elsar_status_string(elsar_status s) {
  switch (s) {
    case ELSAR_OK: return "ok";
    case ELSAR_E_INVALID_ARG: return "invalid argument";
    case ELSAR_E_NO_MEMORY: return "workspace too small or allocation failed";
    case ELSAR_E_HIP: return "HIP runtime error";
    case ELSAR_E_UNSUPPORTED: return "unsupported shape";
    case ELSAR_E_MODEL_REJECTED: return "learned model rejected; RMI kept";
  }
  return "unknown status";
}

}  // extern "C"
