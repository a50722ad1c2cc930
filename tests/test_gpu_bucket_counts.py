"""GPU parity of the bookkeeping scans at bucket counts around their block
decomposition.  Below 16384 buckets the region sizes and the offset scan run
in one block that gives each wave a contiguous segment of buckets, walked
256 at a time, four buckets per lane; from 16384 up they run in two launches
over chunks of 4096 buckets, one block each, the second adding the sums of
the chunks ahead.  Bucket counts that are not multiples of four, that end
just before or after a segment, a step or a chunk, and the largest bucket
count, must all give the offsets (Section 3.5's exclusive sums) that the
oracle computes from the same bucket function, the same largest bucket and
mid/big bucket tallies, and a byte-exact sort."""
import numpy as np
import pytest

import datagen
import oracle

R = 100
SMALL_CAP, MID_CAP = 2048, 6144  # buckets above these go to the larger sorts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2305_05671_amd as elsar
    assert torch.cuda.is_available()
    return torch, elsar


@pytest.mark.parametrize("law,n,B", [
    ("skewed", 300_000, 3),          # three buckets of about 10^5: all big
    ("uniform", 300_000, 255),       # one step, a partial lane group at the end
    ("skewed", 300_000, 257),        # one bucket into a second step
    ("uniform", 300_000, 1023),      # one segment less one bucket
    ("mixed", 300_000, 1025),        # one bucket into the second wave's segment
    ("uniform", 300_000, 16_383),    # every wave busy, the last one short
    ("skewed", 400_000, 16_384),     # the smallest chunked count: four full chunks
    ("zipf", 300_000, 16_385),       # a fifth chunk of one bucket
    ("mixed", 300_000, 20_479),      # the last chunk one bucket short
    ("uniform", 400_000, 65_537),
    ("skewed", 300_000, 1 << 21),    # the largest bucket count; most buckets empty
])
def test_offsets_and_tallies_at_segment_edges(env, law, n, B):
    torch, elsar = env
    recs = datagen.generate(datagen.spec(law, seed=B % 97), n)
    print(f"bucket-count case: {law} n={n} B={B}", flush=True)
    d = torch.from_numpy(np.ascontiguousarray(recs).reshape(-1)).to("cuda")
    m = elsar.Model(n, elsar.fit_params(num_buckets=B, seed=7, kind=elsar.RMI))
    m.sample_fit(d)
    part, offsets = m.partition(d)
    torch.cuda.synchronize()
    info = m.info()
    assert info.num_buckets == B
    # the oracle's FP32 evaluation of the GPU's own parameters
    ref = oracle.RMI(info.num_leaves, B)
    ref.root[:] = [info.root_a0, info.root_a1]
    ref.base[:], ref.c[:], ref.b[:], ref.lo[:], ref.hi[:] = m.leaves()
    counts, want = oracle.counts_offsets(ref.buckets(recs), B)
    got = offsets.cpu().numpy().astype(np.uint64)
    assert got.shape == want.shape and got[-1] == n
    if not np.array_equal(got, want):
        bad = np.nonzero(got != want)[0]
        raise AssertionError(f"{bad.size} offsets differ, first at bucket {bad[0]}")
    st = m.partition_stats(part)
    mid = (counts > SMALL_CAP) & (counts <= MID_CAP)
    big = counts > MID_CAP
    assert st.n == n and st.num_buckets == B
    assert st.max_bucket == counts.max()
    assert (st.mid_buckets, st.mid_records) == (int(mid.sum()), int(counts[mid].sum()))
    assert (st.big_buckets, st.big_records) == (int(big.sum()), int(counts[big].sum()))
    out = torch.empty_like(d)
    m.sort_buckets(part, offsets, n, out)
    torch.cuda.synchronize()
    got_recs = out.cpu().numpy().reshape(-1, R)
    want_recs = oracle.sort_records(recs)
    if not np.array_equal(got_recs, want_recs):
        bad = np.nonzero(np.any(got_recs != want_recs, axis=1))[0]
        raise AssertionError(f"{bad.size} records differ, first at output position {bad[0]}")
