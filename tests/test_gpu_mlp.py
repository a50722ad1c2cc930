"""GPU parity of the monotone MLP root against the oracle (oracle/mlp.py).

Forward: the GPU's y (FP32 vector ALUs, bfloat16 matrix cores) against the
FP64 forward with the same bfloat16 rounding points.  Rounding of h1 to
bfloat16 can land on the other side of a tie between FP32 and FP64 (one
bfloat16 ulp, 2^-8 relative, of one hidden unit), which moves y by at most
~64 * max(w3) * max(W2) / 4 * 2^-8; the tolerance below is derived from that.
Gradients: one training step's backward pass against the FP64 backward with
the same rounding points; block-relative error <= 1e-2 on the bfloat16 layer
(W2), <= 1e-4 on the FP32 layers.
The fitted model: leaf ranges equi-depth in the sample, bit-exact against the
oracle; leaves bit-exact against the oracle's spline over them; the trained
root close to the empirical CDF; bucket counts bit-exact against the oracle's
boundary routing; the sort byte-exact.
"""
import numpy as np
import pytest

import datagen
import oracle
from oracle import mlp

R, K = 100, 10

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2305_05671_amd as elsar
    assert torch.cuda.is_available()
    return torch, elsar


def _codes(kind, n, seed, S=20_000):
    recs = datagen.generate(datagen.spec(kind, seed=seed), n)
    return recs, oracle.sample_codes(recs, seed=seed, S=S)


def _params32(P):
    return mlp.pack(P).astype(np.float32)


def _P64(flat32):
    return mlp.unpack(np.asarray(flat32, np.float64))


def _y_tolerance(P):
    # one bfloat16 flip of one h1 unit: 2^-8 * h1 (<= 1) through W2 (times
    # sigmoid' <= 1/4) and w3, summed over the 64 outputs; allow 4 flips per
    # record plus FP32 evaluation error
    return 4 * 64 * P["w3"].max() * P["W2"].max() * 0.25 * 2.0 ** -8 + 1e-5


@pytest.mark.parametrize("scale", [1.0, 8.0])
def test_forward_matches_oracle(env, scale):
    _, elsar = env
    _, codes = _codes("skewed", 200_000, 1)
    q, w = mlp.knots(codes)
    rng = np.random.default_rng(3)
    P = mlp.initial_params(rng.uniform(0, 1, mlp.N_PARAMS))
    P["W2"] *= scale
    P["w3"] *= scale
    flat = _params32(P)
    P = _P64(flat)
    # sorted sample codes, plus codes outside the sample's range and a ragged count
    x = np.concatenate([codes, np.array([0, 1, codes[-1] + 5, 95 ** 8 - 1], np.uint64),
                        rng.choice(codes, 1001)])
    y = elsar.mlp_forward(flat, q, x)
    want = mlp.forward(P, mlp.features(x, q, w), bf16_layer2=True)["y"]
    err = np.abs(y.astype(np.float64) - want)
    tol = _y_tolerance(P)
    assert err.max() <= tol, (err.max(), tol)
    assert np.median(err) <= 1e-5
    # monotone over the sorted sample (exactly up to FP32 evaluation noise)
    ys = y[:codes.size]
    assert np.all(np.diff(ys) >= -1e-6)


def test_gradient_matches_oracle(env):
    _, elsar = env
    _, codes = _codes("zipf", 100_000, 2)
    q, w = mlp.knots(codes)
    rng = np.random.default_rng(5)
    for trial in range(3):
        P = mlp.initial_params(rng.uniform(0, 1, mlp.N_PARAMS))
        P["W2"] *= 1 + 4 * trial
        P["w3"] *= 1 + 10 * trial
        flat = _params32(P)
        P = _P64(flat)
        idx = rng.integers(0, codes.size, elsar.MLP_GRAD_ROWS)
        x = codes[idx]
        t = (idx / codes.size).astype(np.float32)
        loss, g = elsar.mlp_gradient(flat, q, x, t)
        want_loss, want = mlp.loss_and_grads(P, mlp.features(x, q, w), t.astype(np.float64),
                                             bf16_layer2=True, bf16_dz2=True)
        assert loss == pytest.approx(want_loss, rel=1e-4)
        got = mlp.unpack(g.astype(np.float64))
        for k in mlp.PARAM_SHAPES:
            scale = np.abs(want[k]).max()
            rel = np.abs(got[k] - want[k]).max() / max(scale, 1e-30)
            assert rel <= (1e-2 if k == "W2" else 1e-4), (trial, k, rel)


def _fit(env, recs, **kw):
    torch, elsar = env
    d = torch.from_numpy(np.ascontiguousarray(recs).reshape(-1)).to("cuda")
    m = elsar.Model(recs.shape[0], elsar.fit_params(**kw))
    m.sample_fit(d)
    part, offsets = m.partition(d)
    torch.cuda.synchronize()
    return m, part, offsets, d


@pytest.mark.parametrize("kind,n,B,seed", [("skewed", 400_000, 2048, 2), ("zipf", 300_000, 1024, 3)])
def test_fitted_mlp_model(env, kind, n, B, seed):
    _, elsar = env
    recs = datagen.generate(datagen.spec(kind, seed=seed), n)
    # 100 Adam steps: this test also checks how closely training follows the CDF
    m, part, offsets, _ = _fit(env, recs, num_buckets=B, seed=seed, kind=elsar.MLP, accept_ratio=1e9,
                               mlp_steps=100)
    info = m.info()
    assert info.kind_used == elsar.MLP and not m.rejected
    L = info.num_leaves
    assert L == info.mlp_leaves == B  # one equi-depth leaf per bucket by default
    codes = oracle.sample_codes(recs, seed=seed)
    S = codes.size
    params, knots, bound, first = m.mlp()
    q, w = mlp.knots(codes)
    assert np.array_equal(knots, q)
    # leaf ranges: equi-depth in the sorted sample, bit-exact
    assert np.array_equal(first.astype(np.uint64), mlp.equi_depth_first(codes, L))
    # leaves of the GPU's leaf ranges, bit-exact
    ref = oracle.spline_leaves(codes, first.astype(np.uint64), B)
    base, c, b, lo, hi = m.leaves()
    assert np.array_equal(base, ref.base) and np.array_equal(c, ref.c) and np.array_equal(b, ref.b)
    assert np.array_equal(lo, ref.lo) and np.array_equal(hi, ref.hi)
    # boundaries: the code of each leaf's first sample
    assert bound[0] == 0 and bound[L] == np.iinfo(np.uint64).max
    has = first[1:L] < S
    assert np.array_equal(bound[1:L][has], codes[first[1:L][has]])
    # the trained root tracks the empirical CDF, so its guesses land near the
    # sample's own leaf
    y = mlp.forward(_P64(params), mlp.features(codes, q, w), bf16_layer2=True)["y"]
    assert np.sqrt(np.mean((y - np.arange(S) / S) ** 2)) < 0.05
    lv = np.searchsorted(first[:L], np.arange(S), side="right") - 1
    assert np.median(np.abs(mlp.leaf_guess(y, L) - lv)) < 0.05 * L
    # counts bit-exact under the GPU's boundaries (one leaf per bucket: the leaf)
    bk = oracle.routed_leaves(recs, bound)
    _, want = oracle.counts_offsets(bk, B)
    assert np.array_equal(offsets.cpu().numpy().astype(np.uint64), want)
    # Equation 1: bucket ids non-decreasing along the sorted order
    order = oracle.sort_order(recs)
    assert np.all(np.diff(bk[order].astype(np.int64)) >= 0)


def _sort(env, recs, **kw):
    torch, elsar = env
    d = torch.from_numpy(np.ascontiguousarray(recs).reshape(-1)).to("cuda")
    out = elsar.elsar_sort(d, params=elsar.fit_params(**kw))
    torch.cuda.synchronize()
    return out.cpu().numpy().reshape(-1, R)


@pytest.mark.parametrize("kind,n,B,seed", [
    ("skewed", 300_000, 0, 2), ("zipf", 200_000, 256, 3), ("uniform", 250_000, 1024, 4),
    ("staircase", 200_000, 0, 5), ("mixed", 150_000, 4096, 6)])
def test_sort_with_mlp_root_matches_oracle(env, kind, n, B, seed):
    _, elsar = env
    recs = datagen.generate(datagen.spec(kind, seed=seed), n)
    got = _sort(env, recs, num_buckets=B, seed=seed, kind=elsar.MLP, accept_ratio=1e9)
    assert np.array_equal(got, oracle.sort_records(recs))


@pytest.mark.parametrize("n", [2, 100, 1000, 2049, 65_537])
def test_mlp_edge_sizes(env, n):
    _, elsar = env
    recs = datagen.generate(datagen.spec("skewed", seed=n), n)
    for kind in (elsar.MLP, elsar.AUTO):
        got = _sort(env, recs, kind=kind, accept_ratio=1e9)
        assert np.array_equal(got, oracle.sort_records(recs)), kind


def test_rejection_falls_back_to_rmi(env):
    torch, elsar = env
    recs = datagen.generate(datagen.spec("skewed", seed=8), 200_000)
    # a ratio no model can meet: the linear root is kept
    m, part, offsets, d = _fit(env, recs, num_buckets=512, kind=elsar.MLP, accept_ratio=1e-6)
    info = m.info()
    assert m.rejected and info.kind_used == elsar.RMI and info.mlp_rejected == 1
    ref = oracle.RMI(info.num_leaves, 512)
    ref.root[:] = [info.root_a0, info.root_a1]
    ref.base[:], ref.c[:], ref.b[:], ref.lo[:], ref.hi[:] = m.leaves()
    _, want = oracle.counts_offsets(ref.buckets(recs), 512)
    assert np.array_equal(offsets.cpu().numpy().astype(np.uint64), want)
    out = torch.empty_like(d)
    m.sort_buckets(part, offsets, recs.shape[0], out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().reshape(-1, R), oracle.sort_records(recs))
    assert np.array_equal(_sort(env, recs, num_buckets=512, kind=elsar.MLP, accept_ratio=1e-6),
                          oracle.sort_records(recs))


def test_auto_choice(env):
    # uniform keys: the linear root's largest sample bucket is within the
    # acceptance ratio of a perfect model's, so the automatic choice keeps it;
    # skewed keys: it fails, and the spline root takes over
    _, elsar = env
    recs = datagen.generate(datagen.spec("uniform", seed=12), 300_000)
    m, *_ = _fit(env, recs, num_buckets=1024, seed=12, kind=elsar.AUTO)
    assert m.info().kind_used == elsar.RMI and m.info().mlp_rejected == 0
    assert m.info().mlp_leaves == 0  # the equi-depth leaves were not fitted
    with pytest.raises(elsar.ElsarError):
        m.spline()
    recs = datagen.generate(datagen.spec("skewed", seed=13), 300_000)
    m, *_ = _fit(env, recs, num_buckets=1024, seed=13, kind=elsar.AUTO)
    assert m.info().kind_used == elsar.SPLINE and m.info().mlp_leaves == 1024
