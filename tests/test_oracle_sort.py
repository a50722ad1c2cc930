"""Pins for the oracle's sort definition (CPU only).

The oracle sort is the problem statement itself: records ordered by their
leading key bytes in memcmp order (paper, Section 7.1 "Methodology"), equal
keys in input order.  It is checked against things other than itself:
brute force over every permutation of tiny inputs, numpy's stable lexsort on
an equivalent integer key, and invariants that a planted mistake breaks.
"""
import itertools

import numpy as np
import pytest

import datagen
import oracle

R, K = 100, 10


def _tiny(n, n_keys, rng, key_bytes=K, rec=R):
    keys = rng.integers(0, 256, size=(n_keys, key_bytes), dtype=np.uint8)
    recs = rng.integers(0, 256, size=(n, rec), dtype=np.uint8)
    recs[:, :key_bytes] = keys[rng.integers(0, n_keys, size=n)]
    return recs


def _valid(recs, order):
    """Keys non-decreasing in memcmp order, ties by increasing input index."""
    for a, b in zip(order, order[1:]):
        ka, kb = bytes(recs[a, :K]), bytes(recs[b, :K])
        if ka > kb or (ka == kb and a > b):
            return False
    return True


@pytest.mark.parametrize("n", [0, 1, 2, 3, 5, 7])
def test_brute_force_all_permutations(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(4):
        recs = _tiny(n, max(1, min(3, n)), rng)
        valid = [p for p in itertools.permutations(range(n)) if _valid(recs, p)]
        assert len(valid) == 1, "exactly one order satisfies the definition"
        want = recs[list(valid[0])] if n else recs
        got = oracle.sort_records(recs)
        assert np.array_equal(got, want)
        assert list(oracle.sort_order(recs)) == list(valid[0])


def _lexsort_reference(recs):
    """numpy's stable lexsort on (first 8 key bytes big-endian, bytes 8..9, index)."""
    hi = recs[:, :8].copy().view(">u8").ravel().astype(np.uint64)
    lo = (recs[:, 8].astype(np.uint32) << 8) | recs[:, 9].astype(np.uint32)
    idx = np.arange(recs.shape[0])
    return np.lexsort((idx, lo, hi))


@pytest.mark.parametrize("kind", ["uniform", "skewed", "zipf", "staircase"])
def test_matches_library_lexsort(kind):
    recs = datagen.generate(datagen.spec(kind, seed=7), 200_000)
    order = oracle.sort_order(recs)
    assert np.array_equal(order, _lexsort_reference(recs))


def test_arbitrary_bytes_including_nul():
    # memcmp and strncmp differ on 0x00; the oracle must use unsigned memcmp order.
    rng = np.random.default_rng(3)
    recs = _tiny(50_000, 40_000, rng)
    recs[::7, 3] = 0
    recs[::11, 0] = 0xFF
    assert np.array_equal(oracle.sort_order(recs), _lexsort_reference(recs))
    a = np.zeros((2, R), np.uint8)
    a[0, :2] = [0x41, 0x00]
    a[1, :2] = [0x41, 0x80]
    assert list(oracle.sort_order(a)) == [0, 1]


def test_invariants_and_tie_break_from_payload():
    sp = datagen.spec("skewed", seed=11, embed_idx=True)
    recs = datagen.generate(sp, 300_000)
    out = oracle.sort_records(recs)
    assert oracle.first_unsorted(out) == out.shape[0]
    assert oracle.multiset_hash(out) == oracle.multiset_hash(recs)
    idx = np.array([int(bytes(r[K:K + 10])) for r in out])
    keys = out[:, :K]
    same = np.all(keys[1:] == keys[:-1], axis=1)
    assert same.sum() > 1000, "the hot keys give many ties"
    assert np.all(idx[1:][same] > idx[:-1][same]), "ties keep input order"


def test_checkers_fire_on_planted_mistakes():
    recs = datagen.generate(datagen.spec("uniform", seed=5), 20_000)
    out = oracle.sort_records(recs)
    bad = out.copy()
    bad[[100, 101]] = bad[[101, 100]]
    assert oracle.first_unsorted(bad) == 100
    bad = out.copy()
    bad[5, 50] ^= 1
    assert oracle.multiset_hash(bad) != oracle.multiset_hash(recs)
    bad = out.copy()
    bad[7] = bad[8]
    assert oracle.multiset_hash(bad) != oracle.multiset_hash(recs)


def test_stable_order_checker():
    # on records carrying their input index, "strictly increasing (key, index)"
    # holds for the oracle's output and fails exactly where a tie is swapped
    recs = datagen.generate(datagen.spec("skewed", seed=12, embed_idx=True), 200_000)
    out = oracle.sort_records(recs)
    assert oracle.first_unstable(out) == out.shape[0]
    keys = out[:, :K]
    tie = int(np.nonzero(np.all(keys[1:] == keys[:-1], axis=1))[0][0])
    bad = out.copy()
    bad[[tie, tie + 1]] = bad[[tie + 1, tie]]
    assert oracle.first_unsorted(bad) == bad.shape[0]  # the keys alone cannot see it
    assert oracle.first_unstable(bad) == tie
    bad = out.copy()
    bad[[10, 11]] = bad[[11, 10]]
    assert oracle.first_unstable(bad) == 10
    bad = out.copy()
    bad[50] = bad[49]  # a duplicated record: (key, index) repeats
    assert oracle.first_unstable(bad) == 49


def test_rank_of_matches_sorted_position():
    recs = datagen.generate(datagen.spec("skewed", seed=9), 30_000)
    order = oracle.sort_order(recs)
    for pos in [0, 1, 17, 4999, 29_999]:
        i = int(order[pos])
        assert oracle.rank_of_ptr(recs.ctypes.data, recs.shape[0], bytes(recs[i, :K]), i) == pos


def test_parallel_baseline_matches_oracle():
    # the all-core CPU baseline computes the same permutation as the oracle
    recs = datagen.generate(datagen.spec("skewed", seed=13), 100_000)
    perm, used = oracle.parallel_sort_order(recs.ctypes.data, recs.shape[0])
    assert used >= 1
    assert np.array_equal(perm, oracle.sort_order(recs))


def _varlen_records(n, K, lo, seed, alphabet=b"ab\x00\xff"):
    rng = np.random.default_rng(seed)
    recs = rng.integers(0, 256, size=(n, 32), dtype=np.uint8)  # garbage everywhere first
    a = np.frombuffer(alphabet, np.uint8)
    recs[:, :K] = a[rng.integers(0, a.size, size=(n, K))]
    recs[:, lo] = rng.integers(0, K + 3, size=n)  # lengths above K count as K
    return recs


def test_varlen_worked_example():
    # the key is the first len bytes; the rest of the field is ignored padding;
    # a proper prefix sorts first, a 0x00 byte is a byte like any other
    K, lo = 4, 4
    rows = [(b"abXX", 2), (b"ab\x00Y", 3), (b"abc\x00", 3), (b"abZZ", 2), (b"a\xff\xff\xff", 4),
            (b"\x00\x00\x00\x00", 0), (b"ab\x01Q", 3), (b"zzzz", 9)]
    recs = np.zeros((len(rows), 8), np.uint8)
    for i, (k, ln) in enumerate(rows):
        recs[i, :4] = np.frombuffer(k, np.uint8)
        recs[i, lo] = ln
    order = [int(i) for i in oracle.sort_order_varlen(recs, K, lo)]
    # "" < "ab" (twice, input order) < "ab\x00" < "ab\x01" < "abc" < "a\xff\xff\xff" < "zzzz"
    assert order == [5, 0, 3, 1, 6, 2, 4, 7]


@pytest.mark.parametrize("K,lo", [(8, 8), (10, 10), (11, 11), (8, 11)])
def test_varlen_matches_python_bytes_order(K, lo):
    recs = _varlen_records(20_000, K, lo, seed=K + lo)
    lens = np.minimum(recs[:, lo], K)
    want = sorted(range(recs.shape[0]), key=lambda i: (bytes(recs[i, :lens[i]]), i))
    assert [int(x) for x in oracle.sort_order_varlen(recs, K, lo)] == want
