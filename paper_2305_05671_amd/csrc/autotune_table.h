// Records per bucket for batched sorts, indexed by ceil(log2(n)): a job of n
// records gets the largest power of two <= n / kAutotuneRecordsPerBucket[r]
// buckets (at least 1).  Written by paper_2305_05671_amd/autotune.py on
// gfx950: the per-size sweep of whole sorts (uniform and first-byte-Zipf keys,
// the batch workload's two key laws), then the batch-context sweep (the batch
// workload, sorted window by window) over the rows it names; 0 means the
// default, 950.
#pragma once
#include <stdint.h>

namespace elsar {
constexpr uint32_t kAutotuneRows = 33;
constexpr uint32_t kAutotuneRecordsPerBucket[kAutotuneRows] = {
    0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0,
    384, 384, 384, 384, 384, 384, 384, 384, 384, 384, 640,
    640, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
// Partition tiles (256 records) per block in a batch window whose largest job
// has ceil(log2 n) = row; 0 means the default rule (four below 8192 tiles,
// else 2048 blocks).
constexpr uint32_t kAutotunePartTilesPerBlock[kAutotuneRows] = {
    0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0,
    16, 16, 16, 16, 16, 16, 16, 16, 16, 16, 16,
    16, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
}  // namespace elsar
