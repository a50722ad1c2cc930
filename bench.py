#!/usr/bin/env python3
"""Benchmark: ELSAR's hot path (sample + fit, partition, in-bucket sort,
concatenation) on one MI355X, one JSON line on stdout.

Default workload: 100M records x 100 B, uniform printable 10-byte keys, seed 1,
RMI model, 65536 buckets -- the in-HBM sort.  Inputs are synthetic (the shared
seeded generator), resident in HBM before the timed region; every step sorts
the same input into a separate output buffer.

The JSON line carries:
  value          sorted records/s of the whole job
  roofline       the dominant kernel's algorithmic bytes / its mean duration,
                 from HIP events the library records on its launch stream
  cpu_baseline   the oracle (single-threaded qsort of the stable memcmp order)
                 timed on a bounded sample of the same workload on host cores
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
RECORD_BYTES = 100
# Algorithmic bytes per record of each data pass (the method's two passes):
# partition reads and writes every record once, and so does the bucket sort.
PASS_BYTES = 2 * RECORD_BYTES

WORKLOADS = {
    "uniform-100M": dict(kind="uniform", seed=1, n=100_000_000, buckets=65536,
                         desc="100M x 100B, uniform printable 10-byte keys, seed 1, 65536 buckets"),
    "skewed-hot-100M": dict(kind="skewed", seed=2, n=100_000_000, buckets=65536,
                            desc="100M x 100B, per-byte discrete normal keys (mean 'P', sigma 6) with 10% "
                                 "of records on 1000 hot keys, seed 2, 65536 buckets"),
    "uniform-1M": dict(kind="uniform", seed=0, n=1_000_000, buckets=1024,
                       desc="1M x 100B, uniform printable 10-byte keys, seed 0, 1024 buckets"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="uniform-100M", choices=sorted(WORKLOADS))
    ap.add_argument("--model", default="rmi", choices=["rmi", "mlp", "auto"])
    ap.add_argument("--leaves", type=int, default=0, help="RMI leaves L (0: buckets / 16)")
    ap.add_argument("--mlp-steps", type=int, default=0, help="Adam steps of the MLP fit (0: library default)")
    ap.add_argument("--accept-ratio", type=float, default=1.5,
                    help="MLP acceptance: largest sample bucket <= ratio * ideal")
    ap.add_argument("--cpu-records", type=int, default=16_000_000,
                    help="records of the bounded CPU-baseline sample")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain copy kernel of known size (counter calibration)")
    return ap.parse_args()


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2305_05671_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when there is none or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
            if rec.get("source") != source_hash():
                return None
            for name, v in rec["kernels"].items():
                if name.startswith(kernel):
                    return round((v["fetch_GB"] + v["write_GB"]) * 1e9)
    return None


def cpu_baseline(wl, n_cpu):
    import numpy as np

    import datagen
    import oracle

    recs = datagen.generate(datagen.spec(wl["kind"], seed=wl["seed"]), n_cpu)
    oracle.lib()
    t0 = time.perf_counter()
    perm = oracle.sort_order(recs)
    dt = time.perf_counter() - t0
    del perm
    return {"value": n_cpu / dt, "unit": "records/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_cpu} records of the same workload (same generator and seed), "
                      f"single-threaded qsort of record indices by (memcmp key, index), {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    import datagen
    import paper_2305_05671_amd as elsar

    wl = WORKLOADS[args.workload]
    n = wl["n"]
    kind = {"rmi": elsar.RMI, "mlp": elsar.MLP, "auto": elsar.AUTO}[args.model]
    params = elsar.fit_params(num_buckets=wl["buckets"], num_leaves=args.leaves, seed=wl["seed"], kind=kind,
                              mlp_steps=args.mlp_steps, accept_ratio=args.accept_ratio)

    host = torch.empty(n * RECORD_BYTES, dtype=torch.uint8, pin_memory=True)
    datagen.generate_into(datagen.spec(wl["kind"], seed=wl["seed"]), host.data_ptr(), 0, n)
    d_in = host.to("cuda")
    del host
    d_out = torch.empty_like(d_in)
    ws = torch.empty(elsar.sort_workspace_size(n, params), dtype=torch.uint8, device="cuda")
    print(f"bench: {args.workload} resident in HBM ({n * RECORD_BYTES / 1e9:.1f} GB), "
          f"workspace {ws.numel() / 1e9:.1f} GB", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        elsar.elsar_sort(d_in, d_out, params, ws)
    torch.cuda.synchronize()

    elsar.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        elsar.elsar_sort(d_in, d_out, params, ws)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = elsar.timings()
    elsar.set_timing(False)
    ms_per_step = wall / args.steps * 1e3

    # model / partition statistics of one more fit on the same input (outside the timed region)
    m = elsar.Model(n, params)
    m.sample_fit(d_in)
    part, _ = m.partition(d_in)
    st = m.partition_stats(part)
    info = m.info()
    del part, m

    small_records = n - st.mid_records - st.big_records  # records the small-bucket LDS kernel sorts
    kernels = {  # name in the profiles, phase time, algorithmic bytes per launch
        "partition_kernel": (tm.partition_ms, n * PASS_BYTES),
        "bucket_sort_small_kernel": (tm.bucket_sort_lds_ms, small_records * PASS_BYTES),
    }
    dom = max(kernels, key=lambda k: kernels[k][0])
    dur_ms, alg_bytes = kernels[dom]
    achieved = alg_bytes / (dur_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(args.workload, dom), "alg_bytes": alg_bytes,
                "duration_ms": round(dur_ms, 4)}

    result = {
        "metric": "sorted records/s (100-byte records, in-HBM ELSAR sort)",
        "value": n / (ms_per_step * 1e-3),
        "unit": "records/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "records": n, "record_bytes": RECORD_BYTES, "buckets": wl["buckets"],
                   "model": args.model, "model_used": ["rmi", "mlp"][info.kind_used],
                   "leaves": info.num_leaves, "sample": info.sample_size,
                   "max_sample_bucket": info.max_sample_bucket, "ideal_sample_bucket": info.opt_sample_bucket,
                   "parallelism": "single GPU"},
        "algorithmic_GBps": round(2 * PASS_BYTES * n / (ms_per_step * 1e-3) / 1e9, 1),
        "hbm_frac_whole_path": round(2 * PASS_BYTES * n / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "phases_ms": {"sample_fit": round(tm.sample_fit_ms, 3), "partition": round(tm.partition_ms, 3),
                      "scan": round(tm.scan_ms, 3), "bucket_sort_lds": round(tm.bucket_sort_lds_ms, 3),
                      "bucket_sort_rest": round(tm.bucket_sort_rest_ms, 3), "total": round(tm.total_ms, 3)},
        "buckets": {"max": st.max_bucket, "ideal": round(n / st.num_buckets, 1), "spill": st.spill_count,
                    "mid": st.mid_buckets, "big": st.big_buckets, "mid_records": st.mid_records,
                    "big_records": st.big_records},
        "roofline": roofline,
    }
    if args.copy_probe:
        a = torch.empty(n * RECORD_BYTES // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        torch.neg(a, out=b)  # plain copy-shaped kernel: reads and writes n*R bytes
        torch.cuda.synchronize()
        del a, b
    del d_in, d_out, ws
    torch.cuda.empty_cache()
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(wl, min(args.cpu_records, n))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
