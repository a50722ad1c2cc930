"""GPU parity at the full 100M-record size, in the launch configuration the
benchmark times (one elsar_sort call with a caller workspace, 65536 buckets).

The inputs are the benchmark's workloads with every record's input index
written as 10 decimal digits at the start of its payload (the keys, and so
every bucket decision, are the benchmark's own).  The oracle then checks the
whole output in O(n): every adjacent pair has strictly increasing (key,
input index), and the output holds the input's multiset of records (an
order-independent hash).  A permutation of the input sorted strictly by
(key, input index) is unique: it is the stable sort, so these two checks pin
the output byte for byte, ties included (the skewed workload has about 10^7
records on hot keys).  A few input records are also found at the stable rank
the oracle counts for them one by one.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import datagen
import oracle

R, KEY = 100, 10
N, B = 100_000_000, 65536
THREADS, PROBES = 16, 4

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2305_05671_amd as elsar
    assert torch.cuda.is_available()
    return torch, elsar


def _oracle_checks(h_in, h_out, n, seed):
    pin, pout = h_in.data_ptr(), h_out.data_ptr()
    seg = (n + THREADS - 1) // THREADS
    # order per segment, segments overlapping by one record so that every
    # adjacent pair is checked; the hash per disjoint segment (sums commute)
    pairs = [(a, min(n, a + seg + 1)) for a in range(0, n, seg)]
    parts = [(a, min(n, a + seg)) for a in range(0, n, seg)]
    rng = np.random.default_rng(seed)
    idx = [int(i) for i in rng.integers(0, n, PROBES)] + [0, n - 1]
    src, dst = h_in.numpy(), h_out.numpy()
    keys = [bytes(src[i * R:i * R + KEY]) for i in idx]
    with ThreadPoolExecutor(THREADS) as ex:
        unstable = list(ex.map(lambda ab: oracle.first_unstable_ptr(pout + ab[0] * R, ab[1] - ab[0]), pairs))
        h_a = list(ex.map(lambda ab: oracle.multiset_hash_ptr(pin + ab[0] * R, ab[1] - ab[0]), parts))
        h_b = list(ex.map(lambda ab: oracle.multiset_hash_ptr(pout + ab[0] * R, ab[1] - ab[0]), parts))
        ranks = list(ex.map(lambda q: oracle.rank_of_ptr(pin, n, q[0], q[1]), zip(keys, idx)))
    for (a, b), u in zip(pairs, unstable):
        assert u == b - a, f"(key, input index) not strictly increasing at output position {a + u}"
    mask = (1 << 64) - 1
    assert (sum(h_a) & mask) == (sum(h_b) & mask), "output is not a permutation of the input"
    for i, r in zip(idx, ranks):
        assert 0 <= r < n
        assert np.array_equal(src[i * R:(i + 1) * R], dst[r * R:(r + 1) * R]), (
            f"input record {i} is not at its stable rank {r}")


@pytest.mark.parametrize("law,seed,kind_name,ratio", [
    ("uniform", 1, "RMI", 1.5),     # the 100M-record uniform workload the benchmark times
    ("skewed", 2, "AUTO", 1.5),     # the skewed workload with hot keys, automatic root (the spline)
    ("skewed", 2, "MLP", 1e9),      # the same routed by the MLP root (accepted whatever its statistic)
    ("skewed", 2, "RMI", 1.5),      # the same under the linear root (long big-bucket splits)
])
def test_full_size_sort(env, law, seed, kind_name, ratio):
    torch, elsar = env
    print(f"full-size case: {law} seed {seed} root {kind_name}, {N} records", flush=True)
    kind = getattr(elsar, kind_name)
    p = elsar.fit_params(num_buckets=B, seed=seed, kind=kind, accept_ratio=ratio)
    d_in = torch.empty(N * R, dtype=torch.uint8, device="cuda")
    datagen.generate_device(datagen.spec(law, seed=seed, embed_idx=True), d_in.data_ptr(), 0, N,
                            torch.cuda.current_stream().cuda_stream)
    h_in = d_in.cpu()
    d_out = torch.empty_like(d_in)
    ws = torch.empty(elsar.sort_workspace_size(N, p), dtype=torch.uint8, device="cuda")
    elsar.elsar_sort(d_in, d_out, p, ws)
    torch.cuda.synchronize()
    assert torch.equal(d_in[:R * 1000], h_in[:R * 1000].to("cuda")), "the input was modified"
    del ws
    h_out = d_out.cpu()
    del d_in, d_out
    torch.cuda.empty_cache()
    _oracle_checks(h_in, h_out, N, seed)


def test_max_size_sort(env):
    """The largest in-HBM sort the library accepts (ELSAR_MAX_DEVICE_RECORDS,
    4 * 10^8 records): input, output and workspace take about 265 GB of HBM;
    the default bucket count is 2^18.  Checked over the whole output as
    above (key and input index strictly increasing, multiset, probes)."""
    torch, elsar = env
    n = elsar.MAX_DEVICE_RECORDS
    seed = 7
    print(f"max-size case: uniform seed {seed}, {n} records", flush=True)
    p = elsar.fit_params(seed=seed)
    d_in = torch.empty(n * R, dtype=torch.uint8, device="cuda")
    datagen.generate_device(datagen.spec("uniform", seed=seed, embed_idx=True), d_in.data_ptr(), 0, n,
                            torch.cuda.current_stream().cuda_stream)
    d_out = torch.empty_like(d_in)
    ws = torch.empty(elsar.sort_workspace_size(n, p), dtype=torch.uint8, device="cuda")
    elsar.elsar_sort(d_in, d_out, p, ws)
    torch.cuda.synchronize()
    del ws
    h_in = d_in.cpu()
    del d_in
    h_out = d_out.cpu()
    del d_out
    torch.cuda.empty_cache()
    _oracle_checks(h_in, h_out, n, seed)

