"""Pins for the oracle's key encoding, sampler and monotone RMI (CPU only)."""
import math

import numpy as np
import pytest

import datagen
import oracle

R, K = 100, 10


# ------------------------------------------------------------- encoding --

def test_encoding_closed_forms():
    # Section 4: code = sum_i (ASCII(x_i) - 32) * 95^(l-i), here over 8 bytes.
    assert oracle.e8(b" " * 8) == 0
    assert oracle.e8(b"~" * 8) == 95 ** 8 - 1 == 6_634_204_312_890_624
    assert oracle.e8(b"       !") == 1
    assert oracle.e8(b"!       ") == 95 ** 7
    rng = np.random.default_rng(0)
    for _ in range(2000):
        key = bytes(rng.integers(0x20, 0x7F, size=8, dtype=np.uint8))
        want = sum((c - 32) * 95 ** (7 - i) for i, c in enumerate(key))
        assert oracle.e8(key) == want


def test_encoding_capacity_numbers_of_section_4():
    # log2 of sum_{k=1}^{l} 95^k: 59.14 for l = 9, 65.71 for l = 10; 6.37e17
    # partitions; 10-byte records of that many keys are 6369.5 PB.
    s9 = sum(95 ** k for k in range(1, 10))
    s10 = sum(95 ** k for k in range(1, 11))
    assert round(math.log2(s9), 2) == 59.14
    assert round(math.log2(s10), 2) == 65.71
    assert f"{s9:.2e}" == "6.37e+17"
    assert round(s9 * 10 / 1e15, 1) == 6369.5
    # The 8-byte code used here is exact in FP64 (95^8 < 2^53).
    assert 95 ** 8 < 2 ** 53
    top = oracle.e8(b"~" * 8)
    assert int(float(top)) == top


def test_encoding_saturates_outside_printable():
    assert oracle.e8(b"A\x7f" + b" " * 6) == oracle.e8(b"A" + b"~" * 7)
    assert oracle.e8(b"A\x10zzzzzz") == oracle.e8(b"A" + b" " * 7)
    # per-digit clamping would reverse these two; saturation keeps the order
    a, b = b"\x7fz      ", b"\x80a      "
    assert a < b and oracle.e8(a) <= oracle.e8(b)


def test_encoding_monotone_on_arbitrary_bytes():
    rng = np.random.default_rng(1)
    pools = [np.arange(256), np.arange(0x1E, 0x22), np.arange(0x7C, 0x82), np.array([0, 0x20, 0x7E, 0x7F, 0xFF])]
    for pool in pools:
        keys = rng.choice(pool, size=(20_000, 8)).astype(np.uint8)
        keys = keys[np.lexsort(keys.T[::-1])]  # memcmp order
        codes = [oracle.e8(bytes(k)) for k in keys]
        assert all(x <= y for x, y in zip(codes, codes[1:]))


# --------------------------------------------------------------- sampler --

def test_philox_known_answers():
    # Published Philox4x32-10 known-answer vectors.
    assert oracle.philox([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert oracle.philox([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert oracle.philox([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0]) == \
        [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


@pytest.mark.parametrize("n,S", [(1, 1), (500, 500), (50_000, 1024), (1_000_000, 10_000),
                                 (100_000_000, 1_000_000), (2_500_000_000, 10_000_000)])
def test_sample_size(n, S):
    # 1% of the input (Section 3.1), capped at 10M (Section 6), floor 1024, at most n.
    assert oracle.sample_size(n) == S


def test_sample_positions_stratified_and_seeded():
    n, S = 1_000_003, 10_001
    a = oracle.sample_indices(n, S, 5)
    b = oracle.sample_indices(n, S, 5)
    c = oracle.sample_indices(n, S, 6)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    s = np.arange(S, dtype=np.uint64)
    lo, hi = s * n // S, (s + 1) * n // S
    assert np.all(a >= lo) and np.all(a < hi)
    frac = (a - lo) / (hi - lo)
    assert abs(frac.mean() - 0.5) < 0.02 and frac.min() < 0.02 and frac.max() >= 0.98
    assert np.array_equal(oracle.sample_indices(7, 7, 1), np.arange(7))


# ------------------------------------------------------------------- RMI --

def _f32(x):
    return float(np.float32(x))


def test_fit_collinear_points_exact():
    # codes (7s+3)*2^20 are exact in FP32; the target L*s/S is then exactly linear.
    S, L, B = 4096, 16, 256
    s = np.arange(S, dtype=np.uint64)
    codes = (7 * s + 3) << np.uint64(20)
    m = oracle.fit_rmi(codes, L, B)
    a1 = L / (7 * S * 2 ** 20)
    a0 = -3 * L / (7 * S)
    assert m.root[1] == pytest.approx(_f32(a1), rel=1e-6)
    assert m.root[0] == pytest.approx(_f32(a0), rel=1e-6, abs=1e-6)
    # every leaf is an exact line too: target B*s/S on x_l = code - base
    for j in range(L):
        if m.lo[j] == m.hi[j] and m.c[j] == 0:
            continue
        assert m.c[j] == pytest.approx(_f32(B / (7 * S * 2 ** 20)), rel=1e-5)
    # exact line + floor + per-leaf clamps: sample s lands in bucket floor(B*s/S)
    got = np.array([m.bucket_of(int(c)) for c in codes])
    want = (s * B) // S
    assert np.mean(got == want) > 0.99 and np.max(np.abs(got.astype(int) - want.astype(int))) <= 1


def test_fit_root_is_library_least_squares_and_leaves_are_splines():
    recs = datagen.generate(datagen.spec("skewed", seed=3), 200_000)
    codes = oracle.sample_codes(recs, seed=1)
    L, B = 64, 1024
    m = oracle.fit_rmi(codes, L, B)
    S = codes.size
    x = codes.astype(np.float32).astype(np.float64)
    a1, a0 = np.polyfit(x, L * np.arange(S) / S, 1)
    assert m.root[1] == pytest.approx(_f32(max(a1, 0)), rel=1e-6)
    assert m.root[0] == pytest.approx(_f32(a0), rel=1e-5, abs=1e-5)
    leaves = np.array([m.leaf_of(int(c)) for c in codes])
    assert np.all(np.diff(leaves) >= 0)
    checked = 0
    for j in np.unique(leaves):
        sel = np.nonzero(leaves == j)[0]
        f, g = sel[0], sel[-1]
        span = float(np.float32(codes[g] - codes[f]))
        assert m.base[j] == codes[f]
        assert m.b[j] == _f32(B * f / S)
        if span > 0:
            assert m.c[j] == _f32((B * g / S - B * f / S) / span)
            checked += 1
        else:
            assert m.c[j] == 0
        assert m.lo[j] == (B * f) // S and m.hi[j] == min((B * g) // S, B - 1)
        # the spline meets the leaf's bucket range at both ends
        assert m.bucket_of(int(codes[f])) == m.lo[j]
        assert abs(int(m.bucket_of(int(codes[g]))) - int(m.hi[j])) <= 1
    assert checked > 10
    # the leaves refitted under that root reproduce the fit's own leaves, and
    # under another root they follow that root's routing (closed forms above)
    r = oracle.leaves_under_root(codes, float(m.root[0]), float(m.root[1]), L, B)
    for a, b in ((r.base, m.base), (r.c, m.c), (r.b, m.b), (r.lo, m.lo), (r.hi, m.hi)):
        assert np.array_equal(a, b)
    a0, a1 = np.float32(0.5), np.float32(m.root[1] * 0.75)
    r = oracle.leaves_under_root(codes, float(a0), float(a1), L, B)
    lv = np.array([oracle.lib().oracle_rmi_leaf(a0, a1, L, int(c)) for c in codes])
    for j in np.unique(lv):
        sel = np.nonzero(lv == j)[0]
        f, g = sel[0], sel[-1]
        assert r.base[j] == codes[f] and r.b[j] == _f32(B * f / S)
        assert r.lo[j] == (B * f) // S and r.hi[j] == min((B * g) // S, B - 1)


@pytest.mark.parametrize("kind", ["uniform", "skewed", "zipf", "staircase"])
def test_partition_invariant_equation_1(kind):
    # Equation 1: every key of partition j is <= every key of partition j+1.
    recs = datagen.generate(datagen.spec(kind, seed=21), 100_000)
    m = oracle.fit_rmi(oracle.sample_codes(recs, seed=2), 64, 1024)
    assert np.all(m.c >= 0) and m.root[1] >= 0
    assert np.all(m.lo <= m.hi) and np.all(m.hi[:-1] <= m.lo[1:])
    bk = m.buckets(recs)
    assert bk.max() < 1024
    order = oracle.sort_order(recs)
    assert np.all(np.diff(bk[order].astype(np.int64)) >= 0)
    counts, offsets = oracle.counts_offsets(bk, 1024)
    assert counts.sum() == recs.shape[0] and offsets[-1] == recs.shape[0]
    assert np.array_equal(offsets[:-1], np.concatenate([[0], np.cumsum(counts)[:-1]]))


def test_uniform_partitions_are_near_equi_depth():
    # A perfect model gives Poisson(N/B) loads.  A model fitted on a 1% sample
    # (Section 3.1) sees about S/B samples per bucket, so bucket sizes also carry
    # sampling noise of relative size ~ sqrt(B/S); a gap between two samples at a
    # leaf boundary lands in one bucket.
    N, B = 1_000_000, 1024
    recs = datagen.generate(datagen.spec("uniform", seed=0), N)
    codes = oracle.sample_codes(recs, seed=0)
    m = oracle.fit_rmi(codes, 64, B)
    counts, _ = oracle.counts_offsets(m.buckets(recs), B)
    mean = N / B
    rel = math.sqrt(B / codes.size)
    assert counts.std() / mean < 1.5 * rel
    assert counts.max() < mean * (1 + 4 * rel) + math.sqrt(2 * math.log(B) * mean)
    assert counts.min() > 0
    # with a 10x larger sample the same model is much flatter
    codes10 = oracle.sample_codes(recs, seed=0, S=100_000)
    c10, _ = oracle.counts_offsets(oracle.fit_rmi(codes10, 64, B).buckets(recs), B)
    assert c10.std() < 0.6 * counts.std()


def test_degenerate_fits():
    for codes in [np.array([5], np.uint64), np.full(100, 42, np.uint64), np.arange(10, dtype=np.uint64)]:
        for L, B in [(1, 1), (1, 8), (4, 8), (16, 4)]:
            m = oracle.fit_rmi(codes, L, B)
            assert np.all(m.lo <= m.hi) and np.all(m.hi[:-1] <= m.lo[1:]) and m.hi.max() < B
            bk = [m.bucket_of(int(c)) for c in codes]
            assert all(x <= y for x, y in zip(bk, bk[1:]))
    with pytest.raises(ValueError):
        oracle.fit_rmi(np.array([3, 2], np.uint64), 2, 2)


# ------------------------------------------------------ ideal max bucket --

def _brute_opt(runs, B):
    best = None
    n = len(runs)
    for cuts in range(1 << max(0, n - 1)):
        groups, cur = [], runs[0]
        for i in range(1, n):
            if cuts >> (i - 1) & 1:
                groups.append(cur)
                cur = runs[i]
            else:
                cur += runs[i]
        groups.append(cur)
        if len(groups) <= B:
            m = max(groups)
            best = m if best is None else min(best, m)
    return best


def test_opt_max_bucket_brute_force():
    rng = np.random.default_rng(4)
    for _ in range(200):
        runs = list(rng.integers(1, 6, size=rng.integers(1, 9)))
        B = int(rng.integers(1, 6))
        codes = np.repeat(np.arange(len(runs), dtype=np.uint64) * 3, runs)
        assert oracle.opt_max_bucket(codes, B) == _brute_opt(runs, B)


def test_opt_max_bucket_closed_forms():
    assert oracle.opt_max_bucket(np.arange(1000, dtype=np.uint64), 7) == math.ceil(1000 / 7)
    codes = np.concatenate([np.arange(500), np.full(300, 10_000), np.arange(20_000, 20_500)]).astype(np.uint64)
    assert oracle.opt_max_bucket(codes, 64) == 300
