"""What the trained network gains over the method without it.

Skewed keys with hot keys (the c3 law), same seed, same B and L: the
partition under the MLP root against the partition under the linear root.
The gain measured is balance: the largest bucket and the largest sample
bucket.  Both partitions are exact (the sort is checked elsewhere); this test
records what the learned root changes."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


def _stats(torch, elsar, d, n, **kw):
    m = elsar.Model(n, elsar.fit_params(**kw))
    m.sample_fit(d)
    part, offsets = m.partition(d)
    torch.cuda.synchronize()
    st = m.partition_stats(part)
    info = m.info()
    counts = np.diff(offsets.cpu().numpy())
    return st, info, counts


@pytest.mark.parametrize("n,B", [(4_000_000, 4096), (2_000_000, 1024)])
def test_mlp_root_balances_skewed_buckets(n, B):
    import torch
    import paper_2305_05671_amd as elsar
    recs = datagen.generate(datagen.spec("skewed", seed=2), n)
    d = torch.from_numpy(recs.reshape(-1)).to("cuda")
    st_r, info_r, c_r = _stats(torch, elsar, d, n, num_buckets=B, seed=2, kind=elsar.RMI)
    st_m, info_m, c_m = _stats(torch, elsar, d, n, num_buckets=B, seed=2, kind=elsar.MLP, accept_ratio=1e9)
    assert info_r.kind_used == elsar.RMI and info_m.kind_used == elsar.MLP
    ideal = n / B
    cv = lambda c: float(np.std(c) / np.mean(c))
    print(f"\\nn={n} B={B}: largest bucket RMI {st_r.max_bucket} ({st_r.max_bucket / ideal:.1f}x ideal), "
          f"MLP {st_m.max_bucket} ({st_m.max_bucket / ideal:.1f}x); largest sample bucket RMI "
          f"{info_r.max_sample_bucket}, MLP {info_m.max_sample_bucket} (ideal {info_m.opt_sample_bucket}); "
          f"CV RMI {cv(c_r):.2f}, MLP {cv(c_m):.2f}; records in buckets > 6144: RMI {st_r.big_records}, "
          f"MLP {st_m.big_records}")
    assert st_m.max_bucket < st_r.max_bucket
    assert info_m.max_sample_bucket < info_r.max_sample_bucket
