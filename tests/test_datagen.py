"""The shared input generator: determinism, shape and the laws it draws from."""
import numpy as np

import datagen


def test_philox_known_answers():
    assert datagen.philox4x32_10([0, 0, 0, 0], [0, 0]) == [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert datagen.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2) == \
        [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]


def test_deterministic_and_sliceable():
    for kind in ["uniform", "skewed", "zipf", "mixed", "staircase"]:
        sp = datagen.spec(kind, seed=3)
        a = datagen.generate(sp, 10_000)
        assert np.array_equal(a, datagen.generate(sp, 10_000))
        assert np.array_equal(a[2500:7000], datagen.generate(sp, 4500, start=2500))
        assert a.min() >= 0x20 and a.max() <= 0x7E
        assert not np.array_equal(a, datagen.generate(datagen.spec(kind, seed=4), 10_000))


def test_uniform_key_bytes():
    a = datagen.generate(datagen.spec("uniform", seed=0), 200_000)
    h = np.bincount(a[:, :10].ravel() - 0x20, minlength=95)
    assert h.size == 95 and h.min() > 0.9 * h.mean() and h.max() < 1.1 * h.mean()


def test_skewed_law_and_hot_keys():
    thr = datagen.rank_law("normal", 48.0, 6.0)
    p = np.diff(np.concatenate([[0], thr.astype(np.float64)])) / 2 ** 32
    assert abs((p * np.arange(95)).sum() - 48) < 1e-6
    assert abs(np.sqrt((p * (np.arange(95) - 48) ** 2).sum()) - 6) < 0.01
    a = datagen.generate(datagen.spec("skewed", seed=2), 300_000)
    keys = a[:, :10].copy().view("S10").ravel()
    _, cnt = np.unique(keys, return_counts=True)
    dup = cnt[cnt > 5].sum() / a.shape[0]
    assert 0.09 < dup < 0.11, "about 10% of records carry one of the hot keys"
    assert abs(a[:, 0].astype(float).mean() - (0x20 + 48)) < 0.2


def test_zipf_first_byte():
    a = datagen.generate(datagen.spec("zipf", seed=1), 200_000)
    h = np.bincount(a[:, 0] - 0x20, minlength=95) / a.shape[0]
    w = np.arange(1, 96, dtype=float) ** -1.1
    assert abs(h[0] - w[0] / w.sum()) < 0.01 and h[0] > 0.2
    assert np.all(np.diff(h[:5]) < 0)


def test_embedded_index():
    a = datagen.generate(datagen.spec("uniform", seed=1, embed_idx=True), 1000, start=123)
    assert [int(bytes(r[10:20])) for r in a[:3]] == [123, 124, 125]


def test_job_sizes_log_uniform():
    n = datagen.job_sizes(3, 4096)
    assert n.min() >= 1024 and n.max() <= 4 * 2 ** 20
    lg = np.log(n.astype(float))
    assert abs(lg.mean() - (np.log(1024) + np.log(4 * 2 ** 20)) / 2) < 0.1
    assert 1.7e9 < n.sum() < 2.4e9
