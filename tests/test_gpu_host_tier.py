"""GPU parity of the host tier: records in host memory (pinned or pageable),
sorted into host memory through HBM -- sorted runs written once, then group
passes -- byte-exact against the oracle, on random, key-ordered and
half-and-half inputs, with buckets larger than a pass."""
import numpy as np
import pytest

import datagen
import oracle

R = 100
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2305_05671_amd as elsar
    assert torch.cuda.is_available()
    return torch, elsar


def _pinned(torch, recs, pinned=True):
    t = torch.empty(recs.size, dtype=torch.uint8, pin_memory=pinned)
    t.numpy()[:] = recs.reshape(-1)
    return t


@pytest.mark.parametrize("kind,n,chunk,pass_records,B,pinned", [
    ("uniform", 3_000_001, 250_000, 700_000, 0, True),   # several chunks (ragged last), five passes
    ("skewed", 2_000_000, 333_333, 900_000, 0, True),    # hot keys: buckets above the LDS caps inside passes
    ("zipf", 1_500_000, 0, 0, 1024, True),               # one chunk, one pass
    ("mixed", 777_777, 100_000, 250_000, 512, False),    # pageable host memory
    ("uniform", 1_000_000, 30_000, 300_000, 0, False),   # sample from a first chunk smaller than S
])
def test_host_tier_matches_oracle(env, kind, n, chunk, pass_records, B, pinned):
    torch, elsar = env
    recs = datagen.generate(datagen.spec(kind, seed=41), n)
    h_in = _pinned(torch, recs, pinned)
    h_out = torch.zeros_like(h_in)
    if pinned:
        h_out = h_out.pin_memory()
    st = elsar.sort_host(h_in, h_out, elsar.fit_params(num_buckets=B, seed=41), chunk_records=chunk,
                         pass_records=pass_records)
    if pass_records:
        assert st.passes >= n // pass_records
    got = h_out.numpy().reshape(-1, R)
    want = oracle.sort_records(recs)
    assert np.array_equal(got, want)
    # the input is left as it was
    assert np.array_equal(h_in.numpy().reshape(-1, R), recs)


def test_host_tier_mlp_root(env):
    torch, elsar = env
    recs = datagen.generate(datagen.spec("skewed", seed=42), 1_000_000)
    h_in = _pinned(torch, recs)
    h_out = torch.zeros_like(h_in).pin_memory()
    elsar.sort_host(h_in, h_out, elsar.fit_params(kind=elsar.MLP, accept_ratio=1e9, seed=42), chunk_records=300_000,
                    pass_records=400_000)
    assert np.array_equal(h_out.numpy().reshape(-1, R), oracle.sort_records(recs))


@pytest.mark.parametrize("kind_name", ["SPLINE", "AUTO"])
def test_host_tier_spline_root(env, kind_name):
    # the equi-depth root through the counting pass and the filtered placement
    torch, elsar = env
    recs = datagen.generate(datagen.spec("skewed", seed=44), 1_200_000)
    h_in = _pinned(torch, recs)
    h_out = torch.zeros_like(h_in).pin_memory()
    st = elsar.sort_host(h_in, h_out, elsar.fit_params(kind=getattr(elsar, kind_name), seed=44),
                         chunk_records=300_000, pass_records=500_000)
    assert st.passes >= 3
    assert np.array_equal(h_out.numpy().reshape(-1, R), oracle.sort_records(recs))


def _host_sort(env, recs, pinned=True, **kw):
    torch, elsar = env
    h_in = _pinned(torch, recs, pinned)
    h_out = torch.zeros_like(h_in)
    if pinned:
        h_out = h_out.pin_memory()
    params = kw.pop("params", None) or elsar.fit_params(seed=45)
    st = elsar.sort_host(h_in, h_out, params, **kw)
    return st, h_in, h_out


def test_host_tier_bucket_larger_than_a_pass(env):
    # every key equal: one bucket holds everything, more than a pass; it is
    # copied through in run order, which is the input order of equal keys
    torch, elsar = env
    recs = datagen.generate(datagen.spec("uniform", seed=43, embed_idx=True), 200_000)
    recs[:, :10] = np.frombuffer(b"ALLTHESAME", np.uint8)
    st, _, h_out = _host_sort(env, recs, chunk_records=50_000, pass_records=60_000)
    assert st.copy_passes >= 1
    assert np.array_equal(h_out.numpy().reshape(-1, R), oracle.sort_records(recs))
    # with room for it, the same input sorts through a group pass
    st, _, h_out = _host_sort(env, recs, chunk_records=50_000)
    assert st.copy_passes == 0
    assert np.array_equal(h_out.numpy().reshape(-1, R), oracle.sort_records(recs))


def test_host_tier_oversize_bucket_with_different_keys_is_refused(env):
    # 8 equal leading key bytes (one code, so one bucket) with different bytes
    # 8..9 and more records than a pass: no model can split them
    _, elsar = env
    rng = np.random.default_rng(3)
    recs = datagen.generate(datagen.spec("uniform", seed=46), 200_000)
    recs[:, :8] = np.frombuffer(b"SAMEPREF", np.uint8)
    recs[:, 8:10] = rng.integers(0x20, 0x7F, size=(recs.shape[0], 2), dtype=np.uint8)
    with pytest.raises(elsar.ElsarError) as e:
        _host_sort(env, recs, chunk_records=50_000, pass_records=60_000)
    assert e.value.status == elsar.E_UNSUPPORTED


def _ordered(kind, n, seed):
    recs = datagen.generate(datagen.spec("uniform", seed=seed, embed_idx=True), n)
    if kind == "sorted":
        return oracle.sort_records(recs)
    if kind == "reverse":
        return oracle.sort_records(recs)[::-1].copy()
    # contiguous halves: uniform keys, then the skewed law with hot keys
    half = datagen.generate(datagen.spec("skewed", seed=seed + 1, embed_idx=True), n - n // 2, start=n // 2)
    return np.concatenate([recs[:n // 2], half])


@pytest.mark.parametrize("kind", ["sorted", "reverse", "halves"])
@pytest.mark.parametrize("kind_name", ["RMI", "AUTO"])
def test_host_tier_key_ordered_inputs(env, kind, kind_name):
    # key-ordered input larger than a pass: the model's sample spans the whole
    # input, so no bucket outgrows a pass; at least 5 group passes
    _, elsar = env
    n = 1_000_003
    recs = _ordered(kind, n, 47)
    st, _, h_out = _host_sort(env, recs, params=elsar.fit_params(seed=47, kind=getattr(elsar, kind_name)),
                              chunk_records=150_000, pass_records=180_000)
    assert st.passes >= 5 and st.copy_passes == 0 and st.runs == 7
    assert np.array_equal(h_out.numpy().reshape(-1, R), oracle.sort_records(recs))
    # every record crossed the link four times, plus the sample
    assert 4 * n * R <= st.link_bytes <= 4 * n * R + 2 * oracle.sample_size(n) * R


def test_host_tier_first_chunk_sample_on_sorted_input(env):
    # the paper's first-batch sample on sorted input: every later key lands in
    # the last bucket, which outgrows a pass with different keys -- refused;
    # the same call on shuffled input sorts
    _, elsar = env
    n = 600_000
    recs = _ordered("sorted", n, 48)
    with pytest.raises(elsar.ElsarError) as e:
        _host_sort(env, recs, chunk_records=100_000, pass_records=150_000, first_chunk_sample=True)
    assert e.value.status == elsar.E_UNSUPPORTED
    shuffled = recs[np.random.default_rng(0).permutation(n)]
    st, _, h_out = _host_sort(env, shuffled, chunk_records=100_000, pass_records=150_000, first_chunk_sample=True)
    assert np.array_equal(h_out.numpy().reshape(-1, R), oracle.sort_records(shuffled))


def test_host_tier_runs_over_the_input(env):
    # the fragment store may be the input itself: it then holds the sorted runs
    torch, elsar = env
    n, chunk = 500_000, 120_000
    recs = datagen.generate(datagen.spec("zipf", seed=49), n)
    h_in = _pinned(torch, recs)
    h_out = torch.zeros_like(h_in).pin_memory()
    st = elsar.sort_host(h_in, h_out, elsar.fit_params(seed=49), chunk_records=chunk, pass_records=150_000,
                         h_frag=h_in)
    assert st.runs == 5
    assert np.array_equal(h_out.numpy().reshape(-1, R), oracle.sort_records(recs))
    runs = h_in.numpy().reshape(-1, R)
    for a in range(0, n, chunk):
        assert np.array_equal(runs[a:a + chunk], oracle.sort_records(recs[a:a + chunk]))
