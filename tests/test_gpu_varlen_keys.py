"""GPU parity of variable-length keys (Section 4's padding rule) against the
oracle's byte-string comparator: the key of a record is the first len bytes
of its key field, len at record byte key_len_offset; the field's remaining
bytes are padding that must not influence the order; a prefix sorts before
its extensions; equal keys keep input order.  Byte-exact outputs on mixed
lengths with many shared prefixes, under every root, at several key widths
and length positions, with buckets above the LDS caps, through the partition
and sort-buckets calls, and through the host tier."""
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


def _records(n, R, K, lo, seed, alphabet=None):
    """Records with a key of random length in the key field, random bytes
    behind it (padding), the length at byte lo (up to K + 2: over-long values
    count as K), and the input index in the payload."""
    rng = np.random.default_rng(seed)
    recs = datagen.generate(datagen.spec("uniform", seed=seed, record_bytes=R, key_bytes=12, embed_idx=True), n)
    if alphabet is None:
        recs[:, :K] = rng.integers(0x20, 0x7F, size=(n, K), dtype=np.uint8)
    else:
        a = np.frombuffer(alphabet, np.uint8)
        recs[:, :K] = a[rng.integers(0, a.size, size=(n, K))]
    recs[:, lo] = rng.integers(0, K + 3, size=n)
    return recs


def _sort(env, recs, K, lo, **kw):
    torch, elsar = env
    n, R = recs.shape
    d = torch.from_numpy(np.ascontiguousarray(recs).reshape(-1)).to("cuda")
    out = elsar.elsar_sort(d, params=elsar.fit_params(record_bytes=R, key_bytes=K, key_len_offset=lo, **kw))
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(n, R)


def _same(got, want):
    if not np.array_equal(got, want):
        bad = np.nonzero(np.any(got != want, axis=1))[0]
        raise AssertionError(f"{bad.size} records differ, first at output position {bad[0]}")


@pytest.mark.parametrize("kind_name", ["RMI", "SPLINE", "AUTO", "MLP"])
@pytest.mark.parametrize("K,lo,alphabet", [(10, 10, None), (10, 10, b"ab"), (8, 11, b"xy\x00\xff"),
                                           (11, 11, b" !~")])
def test_varlen_sort_matches_oracle(env, kind_name, K, lo, alphabet):
    _, elsar = env
    recs = _records(300_000, 100, K, lo, seed=K * 7 + lo, alphabet=alphabet)
    got = _sort(env, recs, K, lo, num_buckets=1024, kind=getattr(elsar, kind_name), accept_ratio=1e9)
    _same(got, oracle.sort_records_varlen(recs, K, lo))


@pytest.mark.parametrize("n", [1, 2, 3, 1000, 2049, 70_001])
def test_varlen_edge_sizes(env, n):
    recs = _records(n, 100, 10, 10, seed=n, alphabet=b"ab")
    _same(_sort(env, recs, 10, 10), oracle.sort_records_varlen(recs, 10, 10))


def test_varlen_empty_and_full_keys(env):
    # every key empty: all equal, input order, whatever the padding holds;
    # then lengths 0 and K only
    recs = _records(50_000, 100, 10, 10, seed=5)
    recs[:, 10] = 0
    _same(_sort(env, recs, 10, 10), recs)
    recs[::2, 10] = 10
    _same(_sort(env, recs, 10, 10, num_buckets=64), oracle.sort_records_varlen(recs, 10, 10))


@pytest.mark.parametrize("R", [40, 64, 128])
def test_varlen_record_shapes_and_big_buckets(env, R):
    # few distinct keys: buckets far above the LDS caps (split, or LSD passes
    # through global memory for short records)
    recs = _records(200_000, R, 9, 9, seed=R, alphabet=b"ab")
    recs[:, 2:9] = ord("a")
    _same(_sort(env, recs, 9, 9, num_buckets=32), oracle.sort_records_varlen(recs, 9, 9))


def test_varlen_partition_then_sort_buckets(env):
    torch, elsar = env
    recs = _records(250_000, 100, 10, 11, seed=77, alphabet=b"abc\x00")
    d = torch.from_numpy(recs.reshape(-1)).to("cuda")
    m = elsar.Model(recs.shape[0], elsar.fit_params(key_bytes=10, key_len_offset=11, num_buckets=512))
    m.sample_fit(d)
    part, offsets = m.partition(d)
    out = torch.empty_like(d)
    m.sort_buckets(part, offsets, recs.shape[0], out)
    torch.cuda.synchronize()
    want = oracle.sort_records_varlen(recs, 10, 11)
    got = out.cpu().numpy().reshape(-1, 100)
    _same(got, want)
    off = offsets.cpu().numpy()
    for j in (0, 100, 511):
        _same(got[off[j]:off[j + 1]], want[off[j]:off[j + 1]])


def test_varlen_host_tier(env):
    torch, elsar = env
    recs = _records(400_000, 100, 10, 10, seed=78, alphabet=b"abcd")
    h_in = torch.from_numpy(recs.reshape(-1).copy())
    h_out = torch.zeros_like(h_in)
    st = elsar.sort_host(h_in, h_out, elsar.fit_params(key_len_offset=10, seed=3), chunk_records=90_000,
                         pass_records=100_000)
    assert st.passes >= 4
    _same(h_out.numpy().reshape(-1, 100), oracle.sort_records_varlen(recs, 10, 10))


def test_varlen_argument_checks(env):
    torch, elsar = env
    d = torch.zeros(100 * 1000, dtype=torch.uint8, device="cuda")
    for K, lo in [(12, 12), (10, 9), (10, 12)]:
        with pytest.raises(elsar.ElsarError) as e:
            elsar.elsar_sort(d, params=elsar.fit_params(key_bytes=K, key_len_offset=lo))
        assert e.value.status == elsar.E_UNSUPPORTED
    with pytest.raises(elsar.ElsarError) as e:
        elsar.sort_batch([d], params=elsar.fit_params(key_len_offset=10))
    assert e.value.status == elsar.E_UNSUPPORTED
