"""GPU parity of the linear-spline root against the oracle.

The spline root's leaves are equi-depth in the sorted sample (oracle/mlp.py,
equi_depth_first) with the same two-point splines as the RMI's leaves
(oracle.spline_leaves); its K segment knots are the leaves' first codes at
every (i L) / K-th leaf.  A record goes to the leaf whose boundary codes
bracket its code; with one leaf per bucket that leaf is its bucket
(oracle.routed_leaves), otherwise the leaf's line gives the bucket
(oracle.routed_buckets).  The bucket counts are bit-exact and the sort
byte-exact.
"""
import numpy as np
import pytest

import datagen
import oracle
from oracle import mlp

R = 100

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2305_05671_amd as elsar
    assert torch.cuda.is_available()
    return torch, elsar


def _fit(env, recs, **kw):
    torch, elsar = env
    d = torch.from_numpy(np.ascontiguousarray(recs).reshape(-1)).to("cuda")
    m = elsar.Model(recs.shape[0], elsar.fit_params(**kw))
    m.sample_fit(d)
    part, offsets = m.partition(d)
    torch.cuda.synchronize()
    return m, part, offsets, d


@pytest.mark.parametrize("kind,n,B,leaves,seed", [
    ("skewed", 400_000, 2048, 0, 2), ("zipf", 300_000, 1024, 0, 3), ("staircase", 300_000, 1024, 1000, 5),
    ("uniform", 200_000, 256, 40, 4)])
def test_fitted_spline_model(env, kind, n, B, leaves, seed):
    torch, elsar = env
    recs = datagen.generate(datagen.spec(kind, seed=seed), n)
    m, part, offsets, d = _fit(env, recs, num_buckets=B, num_leaves=leaves, seed=seed, kind=elsar.SPLINE)
    info = m.info()
    assert info.kind_used == elsar.SPLINE
    L = info.num_leaves
    assert L == info.mlp_leaves == (leaves or B)  # one leaf per bucket by default
    K = info.spline_segments
    assert K == (L // 64 if L >= 64 else 1)
    codes = oracle.sample_codes(recs, seed=seed)
    knots, bound, first = m.spline()
    assert np.array_equal(first.astype(np.uint64), mlp.equi_depth_first(codes, L))
    ref = oracle.spline_leaves(codes, first.astype(np.uint64), B)
    base, c, b, lo, hi = m.leaves()
    assert np.array_equal(base, ref.base) and np.array_equal(c, ref.c) and np.array_equal(b, ref.b)
    assert np.array_equal(lo, ref.lo) and np.array_equal(hi, ref.hi)
    S = codes.size
    assert np.array_equal(bound, mlp.equi_depth_bound(codes, L))
    assert np.array_equal(knots, bound[(np.arange(K + 1, dtype=np.int64) * L) // K])
    # counts bit-exact under exact routing among the boundaries: with one leaf
    # per bucket the leaf is the bucket, otherwise the leaf's line gives it
    bk = oracle.routed_leaves(recs, bound) if L == B else oracle.routed_buckets(recs, bound, ref)
    _, want = oracle.counts_offsets(bk, B)
    assert np.array_equal(offsets.cpu().numpy().astype(np.uint64), want)
    # Equation 1 along the sorted order
    order = oracle.sort_order(recs)
    assert np.all(np.diff(bk[order].astype(np.int64)) >= 0)
    out = torch.empty_like(d)
    m.sort_buckets(part, offsets, n, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1, R), recs[order])


@pytest.mark.parametrize("kind,n,B,seed", [
    ("skewed", 300_000, 0, 2), ("zipf", 200_000, 256, 3), ("mixed", 150_000, 4096, 6), ("uniform", 100_000, 0, 7),
    ("skewed", 200_000, 1027, 8)])  # a bucket count that is not a multiple of four: the scans' tails
def test_sort_with_spline_root_matches_oracle(env, kind, n, B, seed):
    torch, elsar = env
    recs = datagen.generate(datagen.spec(kind, seed=seed), n)
    d = torch.from_numpy(np.ascontiguousarray(recs).reshape(-1)).to("cuda")
    out = elsar.elsar_sort(d, params=elsar.fit_params(num_buckets=B, seed=seed, kind=elsar.SPLINE))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1, R), oracle.sort_records(recs))


@pytest.mark.parametrize("n", [1, 2, 63, 1000, 2049, 65_537])
def test_spline_edge_sizes(env, n):
    torch, elsar = env
    recs = datagen.generate(datagen.spec("skewed", seed=n), n)
    d = torch.from_numpy(np.ascontiguousarray(recs).reshape(-1)).to("cuda")
    out = elsar.elsar_sort(d, params=elsar.fit_params(seed=n, kind=elsar.SPLINE))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1, R), oracle.sort_records(recs))


def test_spline_all_equal_keys(env):
    # one run of equal codes holding every leaf start: leaf 0 takes the whole
    # run, every other leaf starts after it (empty), at the code + 1
    torch, elsar = env
    recs = datagen.generate(datagen.spec("uniform", seed=9), 50_000)
    recs[:, :10] = np.frombuffer(b"SAMEKEY123", dtype=np.uint8)
    m, part, offsets, d = _fit(env, recs, num_buckets=256, seed=9, kind=elsar.SPLINE)
    knots, bound, first = m.spline()
    codes = oracle.sample_codes(recs, seed=9)
    L = first.size - 1
    assert first[0] == 0 and np.all(first[1:] == codes.size)
    assert np.array_equal(first.astype(np.uint64), mlp.equi_depth_first(codes, L))
    assert np.array_equal(bound, mlp.equi_depth_bound(codes, L))
    out = torch.empty_like(d)
    m.sort_buckets(part, offsets, recs.shape[0], out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1, R), oracle.sort_records(recs))


@pytest.mark.parametrize("n_hot,kind_name,key_bytes", [
    (10, "SPLINE", 10),   # ten hot keys of about 10^4 records: buckets of one key, sorted by input index
    (2, "SPLINE", 10),    # two of about 5 * 10^4: above that kernel's cap, the general split takes them
    (10, "RMI", 10),      # the linear root: big buckets of different keys, handed on after the probe
    (10, "SPLINE", 16),   # keys past 12 bytes: runs of equal 12-byte prefixes finished by the fix-up
])
def test_hot_key_buckets(env, n_hot, kind_name, key_bytes):
    """Heavily repeated keys: under the equi-depth roots each hot key's run of
    sample codes is a leaf (and a bucket) of its own, so its bucket holds that
    one key; the sort is byte-exact whichever kernel takes a big bucket."""
    torch, elsar = env
    n = 1_000_000
    recs = datagen.generate(datagen.spec("skewed", seed=40 + n_hot, n_hot=n_hot, key_bytes=key_bytes), n)
    m, part, offsets, d = _fit(env, recs, num_buckets=1024, seed=41, kind=getattr(elsar, kind_name),
                               key_bytes=key_bytes)
    st = m.partition_stats(part)
    assert st.big_buckets >= n_hot
    if kind_name == "SPLINE":
        # one bucket per hot key holds exactly that key's records
        hot = oracle.e8_records(recs)
        vals, cnt = np.unique(hot, return_counts=True)
        top = np.sort(cnt)[::-1][:n_hot]
        assert st.max_bucket == top[0]
    out = torch.empty_like(d)
    m.sort_buckets(part, offsets, n, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1, R), oracle.sort_records(recs, key_bytes))


@pytest.mark.parametrize("rec_bytes,region_pct", [(48, 0), (100, 1)])
def test_hot_key_buckets_small_records_and_spill(env, rec_bytes, region_pct):
    """The one-key bucket kernel with records below 64 bytes, and with regions
    so small (region_pct 1) that most of each hot key's records sit in the
    spill area."""
    torch, elsar = env
    n = 600_000
    recs = datagen.generate(datagen.spec("skewed", seed=50, n_hot=8, record_bytes=rec_bytes), n)
    m, part, offsets, d = _fit(env, recs, num_buckets=512, seed=51, kind=elsar.SPLINE, record_bytes=rec_bytes,
                               region_pct=region_pct)
    st = m.partition_stats(part)
    assert st.big_buckets >= 8
    if region_pct:
        assert st.spill_count > n // 2
    out = torch.empty_like(d)
    m.sort_buckets(part, offsets, n, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1, rec_bytes), oracle.sort_records(recs))



@pytest.mark.parametrize("fixed,narrow", [(2, 0), (4, 0), (5, 8), (5, 4), (6, 0)])
def test_dense_code_cells(env, fixed, narrow):
    """Keys whose first `fixed` bytes are one constant (and the next one of
    `narrow` values) and whose later bytes follow the clustered law: a narrow
    code range (a small cell shift) with many boundaries per cell, so the
    cell table's sub-tables are built, some with fewer sub-cells than their
    boundaries call for (the shift caps them).  Counts bit-exact under exact
    routing, the sort byte-exact."""
    torch, elsar = env
    # cell shifts 27, 14, 5 (103 of 229 sub-tables capped by it), 3 (253 of
    # 284) and 0 (no sub-table possible)
    n, B = 1_000_000, 4096
    recs = datagen.generate(datagen.spec("skewed", seed=50 + fixed, hot_fraction=0.0, embed_idx=True), n)
    recs[:, :fixed] = np.frombuffer(b"PQRSTUVW"[:fixed], np.uint8)
    if narrow:
        recs[:, fixed] = 0x41 + recs[:, fixed] % narrow
    m, part, offsets, d = _fit(env, recs, num_buckets=B, seed=fixed, kind=elsar.SPLINE)
    assert m.info().kind_used == elsar.SPLINE
    knots, bound, first = m.spline()
    bk = oracle.routed_leaves(recs, bound)
    _, want = oracle.counts_offsets(bk, B)
    assert np.array_equal(offsets.cpu().numpy().astype(np.uint64), want)
    out = torch.empty_like(d)
    m.sort_buckets(part, offsets, n, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1, R), oracle.sort_records(recs))
