"""Seeded synthetic record generator shared by the GPU path's tests/bench and the oracle.

The generator holds none of the sorting method's arithmetic: it only draws
bytes.  Every record is a pure function of (seed, record index) through a
Philox4x32-10 counter-based RNG, so any slice of a data set can be regenerated
on either side and both sides see identical bytes.

Workloads (record = 10-byte printable-ASCII key + 90-byte printable payload, the
record shape of the paper's benchmarks, Section 7.1):

* ``uniform``   -- every key byte iid uniform over 0x20..0x7E.
* ``skewed``    -- every key byte's character rank r in [0, 94] drawn with
  P(r) proportional to exp(-(r-48)^2 / 72) (mean 'P', sigma 6 characters); with
  probability 0.1 a record instead takes one of 1000 hot keys drawn from the same
  law on a separate stream.
* ``zipf``      -- first key byte rank k in 1..95 with P(k) proportional to
  k^-1.1 (byte 0x20+k-1), remaining bytes uniform.
* ``mixed``     -- per record, ``uniform`` with probability 0.5 else ``skewed``.
* ``staircase`` -- uniform records whose first 6 key bytes are replaced by row
  floor(log2(idx)) mod 128 of a 128-row prefix table drawn from our own RNG
  (the paper's one-line description of its skewed data, Section 7.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libelsar_gen.so")
_GPU_LIB_PATH = os.path.join(_HERE, "libelsar_gen_gpu.so")

UNIFORM, NORMAL_HOT, ZIPF_FIRST, MIX, STAIRCASE = 0, 1, 2, 3, 4


class GenSpec(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_uint32),
        ("record_bytes", ctypes.c_uint32),
        ("key_bytes", ctypes.c_uint32),
        ("embed_idx", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("mean_rank", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("hot_fraction", ctypes.c_double),
        ("n_hot", ctypes.c_uint32),
        ("stair_bytes", ctypes.c_uint32),
        ("zipf_s", ctypes.c_double),
        ("mix_p", ctypes.c_double),
    ]


def build(quiet: bool = True) -> str:
    """Compile the generator with gcc (OpenMP) into datagen/libelsar_gen.so."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-Wall",
           "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_gpu(quiet: bool = True) -> str:
    """Compile the GPU generator (gen_gpu.hip, gfx950) into datagen/libelsar_gen_gpu.so."""
    src = os.path.join(_HERE, "gen_gpu.hip")
    tmp = _GPU_LIB_PATH + ".tmp"
    cmd = ["hipcc", "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", tmp, src]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, _GPU_LIB_PATH)
    return _GPU_LIB_PATH


_lib = None
_gpu_lib = None


def gpu_lib():
    global _gpu_lib
    if _gpu_lib is None:
        if not os.path.exists(_GPU_LIB_PATH):
            raise ImportError(f"{_GPU_LIB_PATH} is missing: build it with datagen.build_gpu()")
        L = ctypes.CDLL(_GPU_LIB_PATH)
        L.gen_records_device.argtypes = [ctypes.POINTER(GenSpec), ctypes.POINTER(ctypes.c_uint64),
                                         ctypes.POINTER(ctypes.c_uint64), ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_void_p, ctypes.c_void_p]
        L.gen_records_device.restype = ctypes.c_int
        _gpu_lib = L
    return _gpu_lib


def generate_device(sp: GenSpec, ptr: int, start: int, count: int, stream: int = 0) -> None:
    """Write records start..start+count-1 to device memory at ``ptr`` (same
    bytes as :func:`generate_into`), asynchronously on ``stream``."""
    normal = rank_law("normal", sp.mean_rank, sp.sigma)
    zipf = rank_law("zipf", sp.zipf_s)
    P = ctypes.POINTER(ctypes.c_uint64)
    rc = gpu_lib().gen_records_device(ctypes.byref(sp), normal.ctypes.data_as(P), zipf.ctypes.data_as(P),
                                      start, count, ctypes.c_void_p(ptr), ctypes.c_void_p(stream))
    if rc != 0:
        raise ValueError(f"gen_records_device failed ({rc})")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.gen_records.argtypes = [ctypes.POINTER(GenSpec), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]
        L.gen_records.restype = ctypes.c_int
        L.gen_job_sizes.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.POINTER(ctypes.c_uint64)]
        L.gen_job_sizes.restype = ctypes.c_int
        L.gen_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.gen_philox4x32_10.restype = None
        L.gen_rank_law.argtypes = [ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                   ctypes.POINTER(ctypes.c_uint64)]
        L.gen_rank_law.restype = None
        _lib = L
    return _lib


def spec(kind="uniform", seed=0, record_bytes=100, key_bytes=10, embed_idx=False,
         mean_rank=48.0, sigma=6.0, hot_fraction=0.1, n_hot=1000, zipf_s=1.1, mix_p=0.5,
         stair_bytes=6) -> GenSpec:
    kinds = {"uniform": UNIFORM, "skewed": NORMAL_HOT, "zipf": ZIPF_FIRST, "mixed": MIX,
             "staircase": STAIRCASE}
    k = kinds[kind] if isinstance(kind, str) else int(kind)
    return GenSpec(k, record_bytes, key_bytes, 1 if embed_idx else 0, seed, mean_rank, sigma,
                   hot_fraction, n_hot, stair_bytes, zipf_s, mix_p)


def generate_into(sp: GenSpec, ptr: int, start: int, count: int) -> None:
    """Write records start..start+count-1 to host memory at address ``ptr``."""
    if count == 0:
        return
    rc = lib().gen_records(ctypes.byref(sp), start, count, ctypes.c_void_p(ptr))
    if rc != 0:
        raise ValueError("gen_records rejected the spec")


def generate(sp: GenSpec, n: int, start: int = 0) -> np.ndarray:
    """Return records start..start+n-1 as a (n, record_bytes) uint8 array."""
    out = np.empty((n, sp.record_bytes), dtype=np.uint8)
    generate_into(sp, out.ctypes.data, start, n)
    return out


def job_sizes(seed: int, n_jobs: int, lo: int = 1024, hi: int = 4 * 1024 * 1024) -> np.ndarray:
    out = np.empty(n_jobs, dtype=np.uint64)
    rc = lib().gen_job_sizes(seed, n_jobs, lo, hi, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError("gen_job_sizes rejected its arguments")
    return out


def job_seed(seed: int, j: int) -> int:
    """Per-job seed of a batch: a fixed affine map of (batch seed, job index)."""
    return (seed * 0x100000001B3 + 0x9E3779B97F4A7C15 * (j + 1)) & 0xFFFFFFFFFFFFFFFF


def job_spec(seed: int, j: int) -> GenSpec:
    """Batch workload: even jobs uniform keys, odd jobs Zipf(1.1) first byte."""
    return spec("uniform" if j % 2 == 0 else "zipf", seed=job_seed(seed, j))


def philox4x32_10(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().gen_philox4x32_10(c, k, o)
    return list(o)


def rank_law(which: str, a: float, b: float = 0.0) -> np.ndarray:
    out = np.empty(95, dtype=np.uint64)
    lib().gen_rank_law(0 if which == "normal" else 1, a, b,
                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


# Named workloads: (generator spec kwargs, record count, buckets)
WORKLOADS = {
    "uniform-1M": dict(kind="uniform", seed=0, n=1_000_000, buckets=1024),
    "uniform-100M": dict(kind="uniform", seed=1, n=100_000_000, buckets=65536),
    "skewed-hot-100M": dict(kind="skewed", seed=2, n=100_000_000, buckets=65536),
    "mixed-2.5B": dict(kind="mixed", seed=4, n=2_500_000_000, buckets=1 << 21),
}
BATCH_SEED = 3
BATCH_JOBS = 4096
