"""The GPU record generator writes the same bytes as the host generator."""
import numpy as np
import pytest

import datagen

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["uniform", "skewed", "zipf", "mixed", "staircase"])
@pytest.mark.parametrize("R,K,embed", [(100, 10, False), (100, 10, True), (64, 12, False), (40, 8, False)])
def test_device_generator_matches_host(kind, R, K, embed):
    import torch
    sp = datagen.spec(kind, seed=77, record_bytes=R, key_bytes=K, embed_idx=embed)
    start, n = 123_456_789, 20_011  # ragged count, large indices (staircase rows, digits)
    want = datagen.generate(sp, n, start=start)
    d = torch.empty(n * R, dtype=torch.uint8, device="cuda")
    datagen.generate_device(sp, d.data_ptr(), start, n, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    got = d.cpu().numpy().reshape(n, R)
    assert np.array_equal(got, want)
