"""Bucket-count autotuner for batched sorts.

Two sweeps, both run on the GPU:

* per size (default): whole sorts (elsar_sort, the per-job pipeline of
  elsar_sort_batch) of 2^k records, k in 11..22, over candidate bucket sizes
  (records per bucket), on the batch workload's two key laws (uniform,
  first-byte Zipf); the fastest size per k goes into csrc/autotune_table.h.
* --batch: a batch sorts its jobs window by window (many jobs per launch),
  which changes the trade-off, so this sweep times the batch workload itself
  (bench.py --workload batch-4096) with one value of a knob for every job
  whose ceil(log2 n) is in --rows, rebuilding the library for each candidate,
  and keeps the fastest (0: the default rule).  Knobs: records per bucket
  (--knob rpb), and the partition's tiles per block in a window's launch
  (--knob tiles), a tile shape of the window kernels.

    python -m paper_2305_05671_amd.autotune                          # per-size table
    python -m paper_2305_05671_amd.autotune --batch --rows 11-22     # batch-context table
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


def _body(vals):
    rows = [vals.get(r, 0) for r in range(33)]
    return ",\n    ".join(", ".join(str(v) for v in rows[i:i + 11]) for i in range(0, 33, 11))


def write_table(best, path=TABLE, tiles=None):
    """best: records per bucket by row; tiles: partition tiles per block by
    row (window launches; None keeps the table's current column)."""
    if tiles is None:
        tiles = read_tiles(path) if os.path.exists(path) else {}
    body = _body(best)
    tbody = _body(tiles)
    text = f"""// Records per bucket for batched sorts, indexed by ceil(log2(n)): a job of n
// records gets the largest power of two <= n / kAutotuneRecordsPerBucket[r]
// buckets (at least 1).  Written by paper_2305_05671_amd/autotune.py on
// gfx950: the per-size sweep of whole sorts (uniform and first-byte-Zipf keys,
// the batch workload's two key laws), then the batch-context sweep (the batch
// workload, sorted window by window) over the rows it names; 0 means the
// default, 950.
#pragma once
#include <stdint.h>

namespace elsar {{
constexpr uint32_t kAutotuneRows = 33;
constexpr uint32_t kAutotuneRecordsPerBucket[kAutotuneRows] = {{
    {body}}};
// Partition tiles (256 records) per block in a batch window whose largest job
// has ceil(log2 n) = row; 0 means the default rule (four below 8192 tiles,
// else 2048 blocks).
constexpr uint32_t kAutotunePartTilesPerBlock[kAutotuneRows] = {{
    {tbody}}};
}}  // namespace elsar
"""
    with open(path, "w") as f:
        f.write(text)


def _read(path, name):
    import re
    text = open(path).read()
    key = name + "[kAutotuneRows] = {"
    if key not in text:
        return {}
    body = text[text.index(key) + len(key):]
    vals = [int(v) for v in re.findall(r"\d+", body[:body.index("}")])]
    return {r: v for r, v in enumerate(vals) if v}


def read_table(path=TABLE):
    return _read(path, "kAutotuneRecordsPerBucket")


def read_tiles(path=TABLE):
    return _read(path, "kAutotunePartTilesPerBlock")


def batch_sweep(candidates, jobs=4096, small_rows=range(11, 21), log=sys.stderr, knob="rpb"):
    """Time the batch workload with each candidate for the rows in small_rows
    (the other rows as they are), rebuilding the library each time.  knob:
    "rpb" (records per bucket) or "tiles" (partition tiles per block)."""
    import json
    import subprocess
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2305_05671_amd import _build
    base, tiles = read_table(), read_tiles()
    best, best_ms = None, float("inf")
    for c in candidates:
        t, tl = dict(base), dict(tiles)
        (t if knob == "rpb" else tl).update({r: c for r in small_rows})
        write_table(t, tiles=tl)
        _build.build()
        r = subprocess.run([sys.executable, os.path.join(os.path.dirname(HERE), "bench.py"), "--workload",
                            "batch-4096", "--jobs", str(jobs), "--steps", "3", "--warmup", "1", "--verify-jobs", "2"],
                           capture_output=True, text=True, check=True)
        ms = json.loads(r.stdout.strip().splitlines()[-1])["ms_per_step"]
        what = "records per bucket" if knob == "rpb" else "partition tiles per block"
        print(f"batch, {c} {what} for 2^{small_rows.start}..2^{small_rows.stop - 1}: {ms:.1f} ms",
              file=log, flush=True)
        if ms < best_ms:
            best, best_ms = c, ms
    (base if knob == "rpb" else tiles).update({r: best for r in small_rows})
    write_table(base, tiles=tiles)
    _build.build()
    return base


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kmin", type=int, default=11)
    ap.add_argument("--kmax", type=int, default=22)
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--batch", action="store_true", help="batch-context sweep (rewrites the table in place)")
    ap.add_argument("--candidates", default="0,256,512,768,1200")
    ap.add_argument("--rows", default="11-20", help="table rows (ceil(log2 n)) the batch sweep sets, lo-hi")
    ap.add_argument("--knob", default="rpb", choices=["rpb", "tiles"],
                    help="batch sweep: records per bucket, or partition tiles per block")
    a = ap.parse_args()
    if a.batch:
        lo, hi = (int(x) for x in a.rows.split("-"))
        batch_sweep([int(c) for c in a.candidates.split(",")], small_rows=range(lo, hi + 1), knob=a.knob)
        print(open(TABLE).read())
        return
    write_table(sweep(a.kmin, a.kmax), a.out)
    print(open(a.out).read())


if __name__ == "__main__":
    main()
