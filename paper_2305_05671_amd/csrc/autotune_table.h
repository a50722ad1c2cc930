// Bucket count per job size for batched sorts, indexed by ceil(log2(n)).
// Written by paper_2305_05671_amd/autotune.py from a sweep of whole sorts on
// gfx950 (uniform and first-byte-Zipf keys); rows it did not sweep keep the
// default, the largest power of two <= n / 950.  0 means the default.
#pragma once
#include <stdint.h>

namespace elsar {
constexpr uint32_t kAutotuneRows = 33;
constexpr uint32_t kAutotuneBuckets[kAutotuneRows] = {
    0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0,
    0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
}  // namespace elsar
