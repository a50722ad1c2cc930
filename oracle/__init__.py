"""ORACLE -- test infrastructure only.

A plain, slow, obviously correct CPU implementation of what the GPU sort
computes, used to check it.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package; the product
path (``paper_2305_05671_amd``) never does and shares no code with it.

The C part (``elsar_oracle.c``) holds the sort definition, the key encoding,
the sampler, the RMI fit/evaluation, counts/offsets, the ideal-bucket bound and
the checkers.  ``mlp.py`` holds the FP64 monotone-MLP forward/backward.  Each
function cites the passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libelsar_oracle.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_f32p = ctypes.POINTER(ctypes.c_float)


def build(quiet: bool = True) -> str:
    """Compile the oracle with gcc.  No fast-math, no FMA contraction: the
    FP32 evaluation spec must round exactly as written."""
    src = os.path.join(_HERE, "elsar_oracle.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-Wall",
           "-ffp-contract=off", "-fno-fast-math", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_PAR_PATH = os.path.join(_HERE, "libelsar_oracle_par.so")


def build_parallel(quiet: bool = True) -> str:
    """Compile the all-core CPU baseline (libstdc++ parallel mode, OpenMP)."""
    src = os.path.join(_HERE, "parallel_sort.cpp")
    tmp = _PAR_PATH + ".tmp"
    cmd = ["g++", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c++17", "-Wall", "-o", tmp, src]
    subprocess.run(cmd, check=True, capture_output=quiet)
    os.replace(tmp, _PAR_PATH)
    return _PAR_PATH


_par = None


def parallel_sort_order(recs_ptr: int, n: int, record_bytes: int = 100, key_bytes: int = 10, threads: int = 0):
    """All-core baseline: the stable memcmp-key order by libstdc++'s parallel
    stable sort.  Returns (perm, threads used)."""
    global _par
    if _par is None:
        if not os.path.exists(_PAR_PATH):
            build_parallel()
        _par = ctypes.CDLL(_PAR_PATH)
        _par.oracle_parallel_sort_order.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _u64p,
                                                    ctypes.c_int]
        _par.oracle_parallel_sort_order.restype = ctypes.c_int
    perm = np.empty(n, dtype=np.uint64)
    used = _par.oracle_parallel_sort_order(ctypes.cast(recs_ptr, _u8p), n, record_bytes, key_bytes,
                                           _p(perm, _u64p), threads)
    return perm, int(used)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        sig = {
            "oracle_sort_order": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _u64p], ctypes.c_int),
            "oracle_sort_records": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _u8p], ctypes.c_int),
            "oracle_sort_order_varlen": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                          _u64p], ctypes.c_int),
            "oracle_first_unsorted": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32], ctypes.c_uint64),
            "oracle_first_unstable": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32], ctypes.c_uint64),
            "oracle_multiset_hash": ([_u8p, ctypes.c_uint64, ctypes.c_uint32], ctypes.c_uint64),
            "oracle_rank_of": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _u8p, ctypes.c_uint64],
                               ctypes.c_uint64),
            "oracle_e8": ([_u8p], ctypes.c_uint64),
            "oracle_e8_records": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, _u64p], None),
            "oracle_philox": ([_u32p, _u32p, _u32p], None),
            "oracle_sample_size": ([ctypes.c_uint64], ctypes.c_uint64),
            "oracle_sample_indices": ([ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, _u64p], None),
            "oracle_sample_codes": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                     _u64p], None),
            "oracle_rmi_leaf": ([ctypes.c_float, ctypes.c_float, ctypes.c_uint32, ctypes.c_uint64], ctypes.c_uint32),
            "oracle_leaf_bucket": ([ctypes.c_uint64, ctypes.c_float, ctypes.c_float, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_uint64], ctypes.c_uint32),
            "oracle_fit_rmi": ([_u64p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _f32p, _u64p, _f32p,
                                _f32p, _u32p, _u32p], ctypes.c_int),
            "oracle_rmi_buckets": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, _f32p, ctypes.c_uint32, _u64p, _f32p,
                                    _f32p, _u32p, _u32p, _u32p], None),
            "oracle_spline_leaves": ([_u64p, ctypes.c_uint64, _u64p, ctypes.c_uint32, ctypes.c_uint32, _u64p,
                                      _f32p, _f32p, _u32p, _u32p], None),
            "oracle_routed_buckets": ([_u8p, ctypes.c_uint64, ctypes.c_uint32, _u64p, ctypes.c_uint32, _u64p,
                                       _f32p, _f32p, _u32p, _u32p, _u32p], None),
            "oracle_rmi_buckets_codes": ([_u64p, ctypes.c_uint64, _f32p, ctypes.c_uint32, _u64p, _f32p, _f32p,
                                          _u32p, _u32p, _u32p], None),
            "oracle_leaves_under_root": ([_u64p, ctypes.c_uint64, ctypes.c_float, ctypes.c_float, ctypes.c_uint32,
                                          ctypes.c_uint32, _u64p, _f32p, _f32p, _u32p, _u32p], None),
            "oracle_counts_offsets": ([_u32p, ctypes.c_uint64, ctypes.c_uint32, _u64p, _u64p], ctypes.c_int),
            "oracle_opt_max_bucket": ([_u64p, ctypes.c_uint64, ctypes.c_uint64], ctypes.c_uint64),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _records(recs: np.ndarray) -> np.ndarray:
    recs = np.ascontiguousarray(recs, dtype=np.uint8)
    if recs.ndim != 2:
        raise ValueError("records must be a (n, record_bytes) uint8 array")
    return recs


# ---------------------------------------------------------------- the sort --

def sort_order(recs: np.ndarray, key_bytes: int = 10) -> np.ndarray:
    """Input index of each output position of the stable memcmp-key sort."""
    recs = _records(recs)
    n, R = recs.shape
    perm = np.empty(n, dtype=np.uint64)
    if lib().oracle_sort_order(_p(recs, _u8p), n, R, key_bytes, _p(perm, _u64p)) != 0:
        raise ValueError("bad arguments")
    return perm


def sort_records(recs: np.ndarray, key_bytes: int = 10) -> np.ndarray:
    """Records sorted by (key bytes in memcmp order, input index)."""
    recs = _records(recs)
    n, R = recs.shape
    out = np.empty_like(recs)
    if lib().oracle_sort_records(_p(recs, _u8p), n, R, key_bytes, _p(out, _u8p)) != 0:
        raise ValueError("bad arguments")
    return out


def sort_order_varlen(recs: np.ndarray, key_bytes: int, len_offset: int) -> np.ndarray:
    """Variable-length keys: input index of each output position when the key
    of a record is the first min(record[len_offset], key_bytes) bytes of its
    key field, ordered as byte strings (a prefix first), ties by input index."""
    recs = _records(recs)
    n, R = recs.shape
    perm = np.empty(n, dtype=np.uint64)
    if lib().oracle_sort_order_varlen(_p(recs, _u8p), n, R, key_bytes, len_offset, _p(perm, _u64p)) != 0:
        raise ValueError("bad arguments")
    return perm


def sort_records_varlen(recs: np.ndarray, key_bytes: int, len_offset: int) -> np.ndarray:
    recs = _records(recs)
    return recs[sort_order_varlen(recs, key_bytes, len_offset).astype(np.int64)]


def first_unsorted(recs: np.ndarray, key_bytes: int = 10) -> int:
    recs = _records(recs)
    return int(lib().oracle_first_unsorted(_p(recs, _u8p), recs.shape[0], recs.shape[1], key_bytes))


def first_unsorted_ptr(ptr: int, n: int, record_bytes: int = 100, key_bytes: int = 10) -> int:
    return int(lib().oracle_first_unsorted(ctypes.cast(ptr, _u8p), n, record_bytes, key_bytes))


def first_unstable_ptr(ptr: int, n: int, record_bytes: int = 100, key_bytes: int = 10) -> int:
    """Records carrying their input index as 10 decimal digits after the key:
    first position whose (key, index) is not strictly below the next one's,
    or n."""
    return int(lib().oracle_first_unstable(ctypes.cast(ptr, _u8p), n, record_bytes, key_bytes))


def first_unstable(recs: np.ndarray, key_bytes: int = 10) -> int:
    recs = _records(recs)
    return first_unstable_ptr(recs.ctypes.data, recs.shape[0], recs.shape[1], key_bytes)


def multiset_hash(recs: np.ndarray) -> int:
    recs = _records(recs)
    return int(lib().oracle_multiset_hash(_p(recs, _u8p), recs.shape[0], recs.shape[1]))


def multiset_hash_ptr(ptr: int, n: int, record_bytes: int = 100) -> int:
    return int(lib().oracle_multiset_hash(ctypes.cast(ptr, _u8p), n, record_bytes))


def rank_of_ptr(ptr: int, n: int, key: bytes, idx: int, record_bytes: int = 100, key_bytes: int = 10) -> int:
    k = np.frombuffer(bytes(key), dtype=np.uint8).copy()
    return int(lib().oracle_rank_of(ctypes.cast(ptr, _u8p), n, record_bytes, key_bytes, _p(k, _u8p), idx))


# ---------------------------------------------------------- the encoding --

def e8(key: bytes) -> int:
    k = np.frombuffer(bytes(key[:8]).ljust(8, b"\x00"), dtype=np.uint8).copy()
    return int(lib().oracle_e8(_p(k, _u8p)))


def e8_records(recs: np.ndarray) -> np.ndarray:
    recs = _records(recs)
    out = np.empty(recs.shape[0], dtype=np.uint64)
    lib().oracle_e8_records(_p(recs, _u8p), recs.shape[0], recs.shape[1], _p(out, _u64p))
    return out


# -------------------------------------------------------------- the sample --

def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox(c, k, o)
    return list(o)


def sample_size(n: int) -> int:
    return int(lib().oracle_sample_size(n))


def sample_indices(n: int, S: int, seed: int) -> np.ndarray:
    out = np.empty(S, dtype=np.uint64)
    lib().oracle_sample_indices(n, S, seed, _p(out, _u64p))
    return out


def sample_codes(recs: np.ndarray, seed: int, S: int | None = None) -> np.ndarray:
    """Sorted codes of the sampled keys."""
    recs = _records(recs)
    n, R = recs.shape
    if S is None:
        S = sample_size(n)
    out = np.empty(S, dtype=np.uint64)
    lib().oracle_sample_codes(_p(recs, _u8p), n, R, S, seed, _p(out, _u64p))
    return out


# ----------------------------------------------------------------- the RMI --

class RMI:
    """Monotone two-level RMI parameters (FP32 evaluation spec)."""

    def __init__(self, L: int, B: int):
        self.L, self.B = L, B
        self.root = np.zeros(2, dtype=np.float32)       # a0, a1
        self.base = np.zeros(L, dtype=np.uint64)
        self.c = np.zeros(L, dtype=np.float32)
        self.b = np.zeros(L, dtype=np.float32)
        self.lo = np.zeros(L, dtype=np.uint32)
        self.hi = np.zeros(L, dtype=np.uint32)

    def leaf_of(self, code: int) -> int:
        return int(lib().oracle_rmi_leaf(float(self.root[0]), float(self.root[1]), self.L, int(code)))

    def bucket_of(self, code: int) -> int:
        j = self.leaf_of(code)
        return int(lib().oracle_leaf_bucket(int(self.base[j]), float(self.c[j]), float(self.b[j]),
                                            int(self.lo[j]), int(self.hi[j]), int(code)))

    def buckets_of_codes(self, codes: np.ndarray) -> np.ndarray:
        codes = np.ascontiguousarray(codes, dtype=np.uint64)
        out = np.empty(codes.size, dtype=np.uint32)
        lib().oracle_rmi_buckets_codes(_p(codes, _u64p), codes.size, _p(self.root, _f32p), self.L,
                                       _p(self.base, _u64p), _p(self.c, _f32p), _p(self.b, _f32p),
                                       _p(self.lo, _u32p), _p(self.hi, _u32p), _p(out, _u32p))
        return out

    def buckets(self, recs: np.ndarray) -> np.ndarray:
        recs = _records(recs)
        out = np.empty(recs.shape[0], dtype=np.uint32)
        lib().oracle_rmi_buckets(_p(recs, _u8p), recs.shape[0], recs.shape[1], _p(self.root, _f32p), self.L,
                                 _p(self.base, _u64p), _p(self.c, _f32p), _p(self.b, _f32p),
                                 _p(self.lo, _u32p), _p(self.hi, _u32p), _p(out, _u32p))
        return out


def fit_rmi(codes: np.ndarray, L: int, B: int) -> RMI:
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    m = RMI(L, B)
    rc = lib().oracle_fit_rmi(_p(codes, _u64p), codes.size, L, B, _p(m.root, _f32p), _p(m.base, _u64p),
                              _p(m.c, _f32p), _p(m.b, _f32p), _p(m.lo, _u32p), _p(m.hi, _u32p))
    if rc != 0:
        raise ValueError("fit_rmi: codes must be sorted and S, L, B > 0")
    return m


def leaves_under_root(codes: np.ndarray, a0: float, a1: float, L: int, B: int) -> RMI:
    """The RMI whose root is the given (a0, a1) and whose leaves are fitted
    over the sorted sample as routed by that root (the leaf step of
    fit_rmi)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    m = RMI(L, B)
    m.root[:] = [a0, a1]
    lib().oracle_leaves_under_root(_p(codes, _u64p), codes.size, float(m.root[0]), float(m.root[1]), L, B,
                                   _p(m.base, _u64p), _p(m.c, _f32p), _p(m.b, _f32p), _p(m.lo, _u32p),
                                   _p(m.hi, _u32p))
    return m


def spline_leaves(codes: np.ndarray, first: np.ndarray, B: int) -> RMI:
    """Leaves over given ranges of the sorted sample: leaf j holds samples
    first[j] .. first[j+1]-1 (len(first) = L + 1, first[L] = S).  The returned
    RMI's root fields are unused."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    first = np.ascontiguousarray(first, dtype=np.uint64)
    L = first.size - 1
    if L < 1 or first[-1] != codes.size or np.any(np.diff(first.astype(np.int64)) < 0):
        raise ValueError("first must be non-decreasing with first[L] = S")
    m = RMI(L, B)
    lib().oracle_spline_leaves(_p(codes, _u64p), codes.size, _p(first, _u64p), L, B, _p(m.base, _u64p),
                               _p(m.c, _f32p), _p(m.b, _f32p), _p(m.lo, _u32p), _p(m.hi, _u32p))
    return m


def routed_buckets(recs: np.ndarray, bound: np.ndarray, leaves: RMI) -> np.ndarray:
    """Bucket of every record with the leaf found among boundary codes (leaf j
    takes codes in [bound[j], bound[j+1])) and the leaf's FP32 line."""
    recs = _records(recs)
    bound = np.ascontiguousarray(bound, dtype=np.uint64)
    out = np.empty(recs.shape[0], dtype=np.uint32)
    lib().oracle_routed_buckets(_p(recs, _u8p), recs.shape[0], recs.shape[1], _p(bound, _u64p), leaves.L,
                                _p(leaves.base, _u64p), _p(leaves.c, _f32p), _p(leaves.b, _f32p),
                                _p(leaves.lo, _u32p), _p(leaves.hi, _u32p), _p(out, _u32p))
    return out


def routed_leaves(recs: np.ndarray, bound: np.ndarray) -> np.ndarray:
    """Leaf of every record among boundary codes: the last j with
    bound[j] <= code (leaf j takes codes in [bound[j], bound[j+1]); equal
    boundaries leave the earlier leaves empty).  With one equi-depth leaf per
    bucket this is the bucket, floor(B * the linear spline's CDF)."""
    codes = e8_records(recs)
    b = np.ascontiguousarray(bound, dtype=np.uint64)
    L = b.size - 1
    return (np.searchsorted(b[:L], codes, side="right") - 1).astype(np.uint32)


def counts_offsets(buckets: np.ndarray, B: int):
    buckets = np.ascontiguousarray(buckets, dtype=np.uint32)
    counts = np.empty(B, dtype=np.uint64)
    offsets = np.empty(B + 1, dtype=np.uint64)
    if lib().oracle_counts_offsets(_p(buckets, _u32p), buckets.size, B, _p(counts, _u64p),
                                   _p(offsets, _u64p)) != 0:
        raise ValueError("bucket id out of range")
    return counts, offsets


def opt_max_bucket(codes: np.ndarray, B: int) -> int:
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    return int(lib().oracle_opt_max_bucket(_p(codes, _u64p), codes.size, B))


def sample_gate(max_bucket: int, S: int, B: int, ratio: float):
    """The linear root's gate: the largest sample bucket against what a
    perfect model shows on S sample keys, lambda + sqrt(2 ln B lambda) + 1
    with lambda = S / B (about the largest of B Poisson(lambda) counts).
    Returns (passed, perfect)."""
    import math
    lam = S / B
    perfect = lam + math.sqrt(2.0 * math.log(B) * lam) + 1.0
    return max_bucket <= ratio * perfect, perfect


def sample_ideal(codes: np.ndarray, B: int) -> int:
    """The acceptance test's ideal on a sorted sample: max(ceil(S/B), the
    longest run of equal codes), a lower bound of the best largest bucket
    (opt_max_bucket computes that optimum itself)."""
    c = np.asarray(codes, dtype=np.uint64)
    S = c.size
    starts = np.flatnonzero(np.concatenate([[True], c[1:] != c[:-1], [True]]))
    return max(-(-S // B), int(np.diff(starts).max()))
