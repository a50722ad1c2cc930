"""GPU parity of the host tier: records in pinned host memory, sorted into
host memory through HBM in several passes, byte-exact against the oracle."""
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


def test_host_tier_bucket_larger_than_a_pass(env):
    torch, elsar = env
    recs = datagen.generate(datagen.spec("uniform", seed=43), 200_000)
    recs[:, :10] = np.frombuffer(b"ALLTHESAME", np.uint8)  # one bucket holds everything
    h_in = _pinned(torch, recs)
    h_out = torch.zeros_like(h_in).pin_memory()
    with pytest.raises(elsar.ElsarError) as e:
        elsar.sort_host(h_in, h_out, elsar.fit_params(), chunk_records=50_000, pass_records=100_000)
    assert e.value.status == elsar.E_NO_MEMORY
    # with room for it, the same input sorts
    elsar.sort_host(h_in, h_out, elsar.fit_params(), chunk_records=50_000)
    assert np.array_equal(h_out.numpy().reshape(-1, R), oracle.sort_records(recs))
