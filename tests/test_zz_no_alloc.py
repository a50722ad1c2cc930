"""elsar_sort_noalloc, the entry point that allocates nothing (its workspace
is the library's fixed per-device scratch), against elsar_sort, the entry
point with a caller workspace: byte-identical output, on two calls in a row
(the second smaller, so stale scratch from the first must not leak in), for
the linear root on uniform keys and the automatic choice on skewed keys; and
both against the oracle."""
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


@pytest.mark.parametrize("law,kind_name,sizes", [("uniform", "RMI", (500_000, 123_457)),
                                                 ("skewed", "AUTO", (300_001, 40_000))])
def test_noalloc_matches_elsar_sort(env, law, kind_name, sizes):
    torch, elsar = env
    p = elsar.fit_params(seed=7, kind=getattr(elsar, kind_name))
    for call, n in enumerate(sizes):
        print(f"no-alloc case: {law} {kind_name} call {call} n={n}", flush=True)
        assert elsar.sort_workspace_size(n, p) <= elsar.NOALLOC_SCRATCH_BYTES
        recs = datagen.generate(datagen.spec(law, seed=100 + call), n)
        d_in = torch.from_numpy(recs.reshape(-1)).to("cuda")
        d_a = torch.empty_like(d_in)
        d_b = torch.empty_like(d_in)
        elsar.elsar_sort_noalloc(d_in, d_a, p)
        elsar.elsar_sort(d_in, d_b, p)
        torch.cuda.synchronize()
        a = d_a.cpu().numpy().reshape(-1, R)
        b = d_b.cpu().numpy().reshape(-1, R)
        assert np.array_equal(a, b), f"call {call}: no-alloc output differs from elsar_sort's"
        assert np.array_equal(a, oracle.sort_records(recs)), f"call {call}: differs from the oracle"


def test_noalloc_in_place_and_too_large(env):
    torch, elsar = env
    p = elsar.fit_params()
    recs = datagen.generate(datagen.spec("zipf", seed=3), 50_000)
    d = torch.from_numpy(recs.reshape(-1)).to("cuda")
    elsar.elsar_sort_noalloc(d, d, p)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy().reshape(-1, R), oracle.sort_records(recs))
    # a size whose workspace exceeds the scratch is refused before any work
    big = 2_000_000
    assert elsar.sort_workspace_size(big, p) > elsar.NOALLOC_SCRATCH_BYTES
    src = torch.empty(big * R, dtype=torch.uint8, device="cuda")
    with pytest.raises(elsar.ElsarError) as ei:
        elsar.elsar_sort_noalloc(src, src, p)
    assert ei.value.status == elsar.E_NO_MEMORY
