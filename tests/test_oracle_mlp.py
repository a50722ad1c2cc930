"""Pins for the oracle's monotone MLP (CPU only): central finite differences,
monotonicity, closed forms of the forward pass and of bfloat16 rounding."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import mlp


def _params(seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    P = {k: rng.normal(0, scale, s) for k, s in mlp.PARAM_SHAPES.items()}
    for k in mlp.NONNEG:
        P[k] = np.abs(P[k])
    return P


def test_parameter_count():
    assert mlp.N_PARAMS == 4801
    P = _params()
    assert np.array_equal(mlp.pack(mlp.unpack(mlp.pack(P))), mlp.pack(P))


def test_gradients_match_central_differences():
    rng = np.random.default_rng(1)
    P = _params(2, 0.5)
    P["w3"] *= 0.05  # output of order 1, so the loss is too
    X = rng.uniform(0, 1, (32, 8))
    t = rng.uniform(0, 1, 32)
    loss, g = mlp.loss_and_grads(P, X, t)
    assert loss < 10
    h = 1e-5
    for k, s in mlp.PARAM_SHAPES.items():
        flat = P[k].ravel()
        for i in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            Pp = {kk: vv.copy() for kk, vv in P.items()}
            Pm = {kk: vv.copy() for kk, vv in P.items()}
            Pp[k].ravel()[i] += h
            Pm[k].ravel()[i] -= h
            num = (mlp.loss_and_grads(Pp, X, t)[0] - mlp.loss_and_grads(Pm, X, t)[0]) / (2 * h)
            # central differences: O(h^2) truncation plus ~eps*loss/h round-off
            assert g[k].ravel()[i] == pytest.approx(num, rel=1e-4, abs=1e-9), (k, i)


def test_forward_closed_form():
    # W2 = 0 and W1 = 0: every unit sees only its bias
    P = {k: np.zeros(s) for k, s in mlp.PARAM_SHAPES.items()}
    P["b2"][:] = np.linspace(-2, 2, mlp.H)
    P["w3"][:] = 0.5
    P["b3"][0] = 0.25
    y = mlp.forward(P, np.random.default_rng(0).uniform(0, 1, (5, 8)))["y"]
    want = 0.5 * (1 / (1 + np.exp(-P["b2"]))).sum() + 0.25
    assert np.allclose(y, want)


def test_monotone_in_the_key():
    recs = datagen.generate(datagen.spec("skewed", seed=3), 50_000)
    codes = np.sort(oracle.e8_records(recs))
    q, w = mlp.knots(codes[::7])
    X = mlp.features(codes, q, w)
    assert np.all(np.diff(X, axis=0) >= 0)
    for seed in range(3):
        y = mlp.forward(_params(seed), X, bf16_layer2=True)["y"]
        assert np.all(np.diff(y) >= -1e-12)


def test_features_closed_form():
    codes = np.arange(0, 9000, 1000, dtype=np.uint64)  # 9 sorted codes
    q, w = mlp.knots(codes)
    assert list(q) == [0, 1000, 2000, 3000, 4000, 5000, 6000, 7000, 8000]
    X = mlp.features(np.array([0, 1500, 8000, 9999], np.uint64), q, w)
    assert np.allclose(X[0], 0) and np.allclose(X[2], 1) and np.allclose(X[3], 1)
    assert np.allclose(X[1], [1, 0.5, 0, 0, 0, 0, 0, 0])


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.1415927])
    r = mlp.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0            # tie rounds to even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6                  # tie rounds to even (up)
    assert r[4] == -2.5 and abs(r[5] - 3.140625) < 1e-12


def test_adam_projection_keeps_weights_nonnegative():
    P = _params(4)
    m = {k: np.zeros_like(v) for k, v in P.items()}
    v = {k: np.zeros_like(x) for k, x in P.items()}
    g = {k: np.ones_like(x) * 10 for k, x in P.items()}
    mlp.adam_step(P, m, v, g, 1, lr=100.0)
    for k in mlp.NONNEG:
        assert P[k].min() >= 0


def test_adam_step_closed_form():
    # Step 1 from zero moments: m = 0.1 g and v = 0.001 g^2, and the bias
    # corrections 1/(1 - 0.9) and 1/(1 - 0.999) give back g and g^2, so every
    # parameter moves by -lr g / (|g| + eps).  Step 2 with gradient h:
    # m = 0.09 g + 0.1 h, v = 0.000999 g^2 + 0.001 h^2, corrected by
    # 1/(1 - 0.81) and 1/(1 - 0.998001).  W1, W2, w3 are then clipped at 0,
    # the biases are not.
    lr, eps = 0.05, 1e-8
    P = {k: np.full(s, 0.02) for k, s in mlp.PARAM_SHAPES.items()}
    P["b1"][:] = -0.02
    m = {k: np.zeros(s) for k, s in mlp.PARAM_SHAPES.items()}
    v = {k: np.zeros(s) for k, s in mlp.PARAM_SHAPES.items()}
    g = {k: np.full(s, 3.0) for k, s in mlp.PARAM_SHAPES.items()}
    g["b2"][:] = -2.0
    g["w3"][:] = 1e-9  # comparable to eps: the step shrinks to lr * g / (g + eps) = lr / 11
    mlp.adam_step(P, m, v, g, 1, lr)
    assert np.allclose(P["W2"], 0.0)                        # 0.02 - 0.05 < 0: clipped
    assert np.allclose(P["b1"], -0.02 - lr * 3 / (3 + eps))  # bias: not clipped
    assert np.allclose(P["b2"], 0.02 + lr * 2 / (2 + eps))
    assert np.allclose(P["w3"], 0.02 - lr * 1e-9 / (1e-9 + eps), rtol=1e-12)
    assert np.allclose(m["W1"], 0.3) and np.allclose(v["W1"], 0.009)
    h = {k: np.full(s, -1.0) for k, s in mlp.PARAM_SHAPES.items()}
    before = {k: x.copy() for k, x in P.items()}
    mlp.adam_step(P, m, v, h, 2, lr)
    m2 = 0.09 * 3 + 0.1 * -1.0
    v2 = 0.000999 * 9 + 0.001 * 1.0
    step = lr * (m2 / (1 - 0.9 ** 2)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + eps)
    assert np.allclose(m["b1"], m2) and np.allclose(v["b1"], v2)
    assert np.allclose(P["b1"], before["b1"] - step, rtol=1e-12, atol=0)
    assert np.allclose(P["W1"], np.maximum(before["W1"] - step, 0.0), rtol=1e-12, atol=0)


def test_gate_helpers():
    # the perfect-model bound: lambda + sqrt(2 ln B lambda) + 1, lambda = S/B
    ok, perf = oracle.sample_gate(30, 16384, 1024, 1.5)
    assert perf == pytest.approx(16 + np.sqrt(2 * np.log(1024) * 16) + 1)
    assert ok == (30 <= 1.5 * perf)
    assert oracle.sample_gate(int(1.5 * perf), 16384, 1024, 1.5)[0]
    assert not oracle.sample_gate(int(1.5 * perf) + 1, 16384, 1024, 1.5)[0]
    # the ideal: ceil(S/B), or a longer run of equal codes; it never exceeds the
    # optimum that brute-force packing finds
    c = np.array([1, 2, 2, 2, 2, 3, 4, 5, 6, 7], np.uint64)
    assert oracle.sample_ideal(c, 5) == 4 and oracle.sample_ideal(c, 2) == 5
    rng = np.random.default_rng(1)
    for _ in range(20):
        c = np.sort(rng.integers(0, 30, rng.integers(1, 200))).astype(np.uint64)
        B = int(rng.integers(1, 40))
        assert oracle.sample_ideal(c, B) <= oracle.opt_max_bucket(c, B)


def test_training_reduces_loss_and_leaves_are_monotone():
    recs = datagen.generate(datagen.spec("skewed", seed=5), 100_000)
    codes = oracle.sample_codes(recs, seed=1, S=20_000)
    q, w = mlp.knots(codes)
    X = mlp.features(codes, q, w)
    t = np.arange(codes.size) / codes.size
    rng = np.random.default_rng(7)
    P = mlp.initial_params(rng.uniform(0, 1, mlp.N_PARAMS))
    m = {k: np.zeros_like(x) for k, x in P.items()}
    v = {k: np.zeros_like(x) for k, x in P.items()}
    l0 = mlp.loss_and_grads(P, X, t)[0]
    for step in range(1, 301):
        idx = rng.integers(0, codes.size, 512)
        _, g = mlp.loss_and_grads(P, X[idx], t[idx])
        mlp.adam_step(P, m, v, g, step, lr=1e-2)
    l1 = mlp.loss_and_grads(P, X, t)[0]
    assert l1 < 0.1 * l0 and l1 < 2e-3
    # the network is monotone, so the router's guesses never decrease along the sorted sample
    lv = mlp.leaf_guess(mlp.forward(P, X)["y"], 256)
    assert np.all(np.diff(lv) >= 0) and lv.min() >= 0 and lv.max() < 256


def test_bf16_backward_close_to_fp64():
    # the rounding points of the matrix-core products move the gradient by
    # about one bfloat16 ulp (2^-8) relative, never more than a few percent
    rng = np.random.default_rng(11)
    P = mlp.initial_params(rng.uniform(0, 1, mlp.N_PARAMS))
    X = rng.uniform(0, 1, (128, 8))
    t = np.sort(rng.uniform(0, 1, 128))
    _, g = mlp.loss_and_grads(P, X, t)
    _, gq = mlp.loss_and_grads(P, X, t, bf16_layer2=True, bf16_dz2=True)
    for k in mlp.PARAM_SHAPES:
        scale = np.abs(g[k]).max()
        assert np.abs(gq[k] - g[k]).max() <= 3e-2 * scale, k


def test_equi_depth_first_worked_example():
    # S = 8, L = 4: leaf j would start at sample 2j.  Samples 0 and 2 lie in
    # the same run (three 1s): leaf 0 takes exactly that run and leaf 1 starts
    # after it, at the 2 (boundary 1 + 1 = 2); the start at sample 4 (code 3)
    # moves back to the first sample of its run
    codes = np.array([1, 1, 1, 2, 3, 3, 4, 5], dtype=np.uint64)
    assert list(mlp.equi_depth_first(codes, 4)) == [0, 3, 4, 6, 8]
    top = np.iinfo(np.uint64).max
    assert list(mlp.equi_depth_bound(codes, 4)) == [0, 2, 3, 4, top]
    # a run holding three starts: its first leaf takes it, the next one is empty
    codes = np.array([7, 9, 9, 9, 9, 9, 9, 12], dtype=np.uint64)
    assert list(mlp.equi_depth_first(codes, 4)) == [0, 1, 7, 7, 8]
    assert list(mlp.equi_depth_bound(codes, 4)) == [0, 9, 10, 10, top]


def test_equi_depth_samples_route_to_their_own_leaf():
    # through the boundaries (last j with bound[j] <= code), every sample
    # reaches the leaf whose range holds it; a run that holds several leaf
    # starts is a leaf of its own
    rng = np.random.default_rng(23)
    for trial in range(40):
        S = int(rng.integers(1, 500))
        L = int(rng.integers(1, 80))
        hi = int(rng.choice([4, 30, 10**9]))
        codes = np.sort(rng.integers(0, hi, size=S)).astype(np.uint64)
        f = mlp.equi_depth_first(codes, L).astype(np.int64)
        bound = mlp.equi_depth_bound(codes, L)
        assert f[0] == 0 and f[-1] == S and np.all(np.diff(f) >= 0)
        routed = np.searchsorted(bound[:L], codes, side="right") - 1
        own = np.searchsorted(f[:L], np.arange(S), side="right") - 1
        assert np.array_equal(routed, own)
        q = (np.arange(L) * S) // L
        for j in range(1, L):
            if codes[q[j]] == codes[q[j - 1]]:
                k = j - 1
                while k > 0 and codes[q[k - 1]] == codes[q[j]]:
                    k -= 1
                rs = int(np.searchsorted(codes, codes[q[j]], side="left"))
                re = int(np.searchsorted(codes, codes[q[j]], side="right"))
                assert f[k] == (rs if k > 0 else 0) and f[k + 1] == re  # the run's own leaf


def test_equi_depth_first_properties():
    rng = np.random.default_rng(21)
    for trial in range(20):
        S = int(rng.integers(1, 400))
        L = int(rng.integers(1, 70))
        # distinct codes: the starts are exactly floor(j S / L), one past it
        # where two leaves would start at the same sample (S < L)
        codes = np.sort(rng.choice(10**9, size=S, replace=False)).astype(np.uint64)
        f = mlp.equi_depth_first(codes, L)
        q = [(j * S) // L for j in range(L)]
        assert list(f) == [q[j] + (1 if j and q[j] == q[j - 1] else 0) for j in range(L)] + [S]
        # many equal codes: every start is a run start (at or before
        # floor(j S / L), or the end of the previous leaf's run), and no run
        # straddles two leaves
        codes = np.sort(rng.integers(0, 6, size=S)).astype(np.uint64)
        f = mlp.equi_depth_first(codes, L).astype(np.int64)
        assert f[-1] == S and np.all(np.diff(f) >= 0)
        for j in range(L):
            q = (j * S) // L
            if j and codes[(j - 1) * S // L] == codes[q]:
                assert f[j] == np.searchsorted(codes, codes[q], side="right")
            else:
                assert f[j] <= q and codes[f[j]] == codes[q]
            assert f[j] == 0 or f[j] == S or codes[f[j] - 1] != codes[f[j]]


def test_spline_leaves_exact_on_linear_codes():
    # codes linear in rank: every leaf's spline is the exact CDF, so the bucket
    # of sample s is floor(B s / S), or one less where B s / S is an integer
    # and the FP32 line lands just below it
    S, B, L = 4096, 64, 8
    codes = (1000 + 7 * np.arange(S)).astype(np.uint64)
    first = np.arange(L + 1, dtype=np.uint64) * (S // L)
    m = oracle.spline_leaves(codes, first, B)
    got = np.array([int(oracle.lib().oracle_leaf_bucket(int(m.base[j]), float(m.c[j]), float(m.b[j]),
                                                         int(m.lo[j]), int(m.hi[j]), int(codes[s])))
                    for s in range(S) for j in [s // (S // L)]])
    want = (B * np.arange(S)) // S
    exact = (B * np.arange(S)) % S == 0
    assert np.all(got[~exact] == want[~exact])
    assert np.all((got[exact] == want[exact]) | (got[exact] == want[exact] - 1))


def test_routed_buckets_equal_root_routing():
    # boundaries read off the linear root's own routing give the same buckets
    recs = datagen.generate(datagen.spec("zipf", seed=6), 30_000)
    codes = oracle.sample_codes(recs, seed=6)
    m = oracle.fit_rmi(codes, 16, 256)
    allc = oracle.e8_records(recs)
    leaf = np.array([m.leaf_of(c) for c in allc])
    bound = np.full(m.L + 1, np.iinfo(np.uint64).max, dtype=np.uint64)
    for j in range(m.L - 1, -1, -1):
        sel = allc[leaf >= j]
        bound[j] = sel.min() if sel.size else bound[j + 1]
    bound[0] = 0
    assert np.array_equal(oracle.routed_buckets(recs, bound, m), m.buckets(recs))


def test_routed_leaves_worked_example():
    # three leaves from boundaries [0, code("C..."), code("C...")] (leaf 1 empty):
    # keys before "C" go to leaf 0, "C" and after to leaf 2
    def rec(key):
        r = np.full(100, ord(" "), dtype=np.uint8)
        r[:len(key)] = np.frombuffer(key, dtype=np.uint8)
        return r
    recs = np.stack([rec(b"A"), rec(b"BZZZZZZZZZ"), rec(b"C"), rec(b"D"), rec(b"~~~~~~~~~~")])
    c = oracle.e8_records(recs[2:3])[0]
    bound = np.array([0, c, c, np.iinfo(np.uint64).max], dtype=np.uint64)
    assert list(oracle.routed_leaves(recs, bound)) == [0, 0, 2, 2, 2]


def test_routed_leaves_equal_single_bucket_leaves():
    # leaves that each map to their own bucket (constant lines) route the same
    recs = datagen.generate(datagen.spec("skewed", seed=17), 20_000)
    codes = oracle.sample_codes(recs, seed=17)
    L = 64
    first = mlp.equi_depth_first(codes, L)
    bound = np.full(L + 1, np.iinfo(np.uint64).max, dtype=np.uint64)
    bound[0] = 0
    has = first[1:L] < codes.size
    bound[1:L][has] = codes[first[1:L][has].astype(np.int64)]
    m = oracle.RMI(L, L)
    m.base[:] = 0
    m.c[:] = 0
    m.b[:] = np.arange(L, dtype=np.float32)
    m.lo[:] = np.arange(L, dtype=np.uint32)
    m.hi[:] = np.arange(L, dtype=np.uint32)
    assert np.array_equal(oracle.routed_leaves(recs, bound), oracle.routed_buckets(recs, bound, m))
