"""Bucket-count autotuner for batched sorts.

Sweeps whole sorts (elsar_sort, the per-job pipeline of elsar_sort_batch) of
2^k records for k in 11..22 over candidate bucket sizes (records per bucket),
on the batch workload's two key laws (uniform, first-byte Zipf), and writes
the fastest size per k into csrc/autotune_table.h.  Run it on the GPU, then
rebuild the library:

    python -m paper_2305_05671_amd.autotune            # writes the table
    python -c "import __graft_entry__ as g; g.build()"
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "csrc", "autotune_table.h")
CANDIDATES = (256, 384, 512, 768, 1024, 1536, 2048)


def sweep(kmin=11, kmax=22, reps=20, log=sys.stderr):
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    import datagen
    import paper_2305_05671_amd as elsar

    best = {}
    for k in range(kmin, kmax + 1):
        n = 1 << k
        times = {}
        for law in ("uniform", "zipf"):
            d = torch.empty(n * 100, dtype=torch.uint8, device="cuda")
            datagen.generate_device(datagen.spec(law, seed=k), d.data_ptr(), 0, n,
                                    torch.cuda.current_stream().cuda_stream)
            out = torch.empty_like(d)
            for per in CANDIDATES:
                B = 1
                while B * 2 * per <= n:
                    B *= 2
                p = elsar.fit_params(num_buckets=B, seed=k)
                ws = torch.empty(elsar.sort_workspace_size(n, p), dtype=torch.uint8, device="cuda")
                for _ in range(3):
                    elsar.elsar_sort(d, out, p, ws)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    elsar.elsar_sort(d, out, p, ws)
                e1.record()
                torch.cuda.synchronize()
                times[per] = times.get(per, 0.0) + e0.elapsed_time(e1) / reps
        per = min(times, key=times.get)
        best[k] = per
        print(f"n=2^{k}: " + ", ".join(f"{q}:{t:.3f}ms" for q, t in sorted(times.items())) + f" -> {per}",
              file=log, flush=True)
    return best


def write_table(best, path=TABLE):
    rows = [best.get(r, 0) for r in range(33)]
    body = ",\n    ".join(", ".join(str(v) for v in rows[i:i + 11]) for i in range(0, 33, 11))
    text = f"""// Records per bucket for batched sorts, indexed by ceil(log2(n)): a job of n
// records gets the largest power of two <= n / kAutotuneRecordsPerBucket[r]
// buckets (at least 1).  Written by paper_2305_05671_amd/autotune.py from a
// sweep of whole sorts on gfx950 (uniform and first-byte-Zipf keys, the
// batch workload's two key laws); 0 means the default, 950.
#pragma once
#include <stdint.h>

namespace elsar {{
constexpr uint32_t kAutotuneRows = 33;
constexpr uint32_t kAutotuneRecordsPerBucket[kAutotuneRows] = {{
    {body}}};
}}  // namespace elsar
"""
    with open(path, "w") as f:
        f.write(text)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kmin", type=int, default=11)
    ap.add_argument("--kmax", type=int, default=22)
    ap.add_argument("--out", default=TABLE)
    a = ap.parse_args()
    write_table(sweep(a.kmin, a.kmax), a.out)
    print(open(a.out).read())


if __name__ == "__main__":
    main()
