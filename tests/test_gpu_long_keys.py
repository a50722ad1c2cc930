"""GPU parity for keys longer than 12 bytes (13..28): the bucket sorts order
key bytes 0..11 and the input index, then runs of equal 12-byte prefixes are
sorted stably by the rest of the key.  Every case is byte-exact against the
oracle's stable memcmp sort over the whole key.

The inputs put many records on few 12-byte prefixes (long runs, sorted through
global memory), many prefixes with a few records each (short runs), suffixes
drawn from a small alphabet (equal suffixes keep input order), and whole-key
duplicates (runs already in order, which the fix-up leaves alone)."""
import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2305_05671_amd as elsar
    assert torch.cuda.is_available()
    return torch, elsar


def _records(n, R, K, n_prefix, alphabet, seed, dup_every=0):
    rng = np.random.default_rng(seed)
    recs = datagen.generate(datagen.spec("uniform", seed=seed, record_bytes=R, key_bytes=10), n)
    prefixes = rng.integers(0x20, 0x7F, size=(n_prefix, 12), dtype=np.uint8)
    recs[:, :12] = prefixes[rng.integers(0, n_prefix, size=n)]
    recs[:, 12:K] = rng.choice(np.frombuffer(alphabet, np.uint8), size=(n, K - 12))
    if dup_every:
        recs[dup_every::dup_every, :K] = recs[0, :K]  # one key many times
    return recs


def _sort(env, recs, R, K, **kw):
    torch, elsar = env
    d = torch.from_numpy(np.ascontiguousarray(recs).reshape(-1)).to("cuda")
    out = elsar.elsar_sort(d, params=elsar.fit_params(record_bytes=R, key_bytes=K, **kw))
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(-1, R)


def _assert_same(got, want):
    assert got.shape == want.shape
    if not np.array_equal(got, want):
        bad = np.nonzero(np.any(got != want, axis=1))[0]
        raise AssertionError(f"{bad.size} records differ, first at output position {bad[0]}")


@pytest.mark.parametrize("kind_name", ["RMI", "SPLINE"])
@pytest.mark.parametrize("K", [13, 16, 20, 27, 28])
def test_long_keys_long_runs(env, K, kind_name):
    # 8 prefixes: runs of about 12 500 records, sorted in several 4096-entry tiles
    _, elsar = env
    recs = _records(100_000, 100, K, 8, b"ABCD", seed=K)
    _assert_same(_sort(env, recs, 100, K, num_buckets=256, kind=getattr(elsar, kind_name)),
                 oracle.sort_records(recs, key_bytes=K))


@pytest.mark.parametrize("K", [14, 24])
def test_long_keys_short_runs_and_duplicates(env, K):
    # 20 000 prefixes (runs of about 10), and one whole key on every 7th record
    recs = _records(200_000, 100, K, 20_000, b"xy", seed=100 + K, dup_every=7)
    _assert_same(_sort(env, recs, 100, K, num_buckets=1024), oracle.sort_records(recs, key_bytes=K))


@pytest.mark.parametrize("R,K", [(40, 28), (128, 17), (64, 21)])
def test_long_keys_record_shapes(env, R, K):
    # keys that fill most of a short record, and key ends inside a dword
    recs = _records(60_000, R, K, 50, b"0123456789", seed=R + K)
    _assert_same(_sort(env, recs, R, K, num_buckets=64), oracle.sort_records(recs, key_bytes=K))


def test_long_keys_uniform_bytes(env):
    # no shared 12-byte prefixes at all: the fix-up finds no run
    recs = datagen.generate(datagen.spec("uniform", seed=5), 300_000)
    rng = np.random.default_rng(5)
    recs[:, :20] = rng.integers(0, 256, size=(recs.shape[0], 20), dtype=np.uint8)
    _assert_same(_sort(env, recs, 100, 20, num_buckets=512), oracle.sort_records(recs, key_bytes=20))


@pytest.mark.parametrize("n", [0, 1, 2, 3, 257])
def test_long_keys_edge_sizes(env, n):
    recs = _records(max(n, 1), 100, 20, 1, b"ab", seed=n)[:n]
    _assert_same(_sort(env, recs, 100, 20, num_buckets=4), oracle.sort_records(recs, key_bytes=20))


def test_long_keys_host_tier(env):
    # several passes and chunks: runs are finished inside each pass's stage
    torch, elsar = env
    recs = _records(600_000, 100, 22, 300, b"pq", seed=22)
    h_in = torch.from_numpy(recs.reshape(-1).copy())
    h_out = torch.zeros_like(h_in)
    st = elsar.sort_host(h_in, h_out, elsar.fit_params(key_bytes=22, num_buckets=512, seed=3),
                         chunk_records=100_000, pass_records=200_000)
    assert st.passes >= 3
    _assert_same(h_out.numpy().reshape(-1, 100), oracle.sort_records(recs, key_bytes=22))


def test_long_keys_batch_rejected(env):
    torch, elsar = env
    d = torch.zeros(100 * 1000, dtype=torch.uint8, device="cuda")
    with pytest.raises(Exception, match="elsar_sort_batch_workspace_size"):
        elsar.sort_batch([d], params=elsar.fit_params(key_bytes=16))
