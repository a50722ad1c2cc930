"""ORACLE -- test infrastructure only: the monotone MLP CDF in FP64.

The paper's model is an RMI of linear regressions (Section 3.1).  The learned
root this build adds is a small monotone MLP fitted to the same target, the
empirical CDF of the sample (rank / S), and used as the RMI's root.  This module
is the plain reference of what the GPU computes: features, forward pass, MSE
loss, backward pass, the Adam step with the non-negativity projection, and the
equi-depth leaf ranges of a sorted sample.  Everything is FP64 numpy; ``bf16=True``
rounds the hidden activations and the 64x64 weights to bfloat16 the way the GPU
feeds its matrix cores, for parity checks on identical inputs.

Architecture (8 -> 64 -> 64 -> 1):
  phi_k(code) = min(1, max(code - q_k, 0) / w_k), k = 0..7, q_k the codes at
                the sample's 1/8 quantiles, w_k = max(q_{k+1} - q_k, 1)
  h1 = sigmoid(W1 phi + b1)      W1 >= 0
  h2 = sigmoid(W2 h1 + b2)       W2 >= 0
  y  = w3 . h2 + b3              w3 >= 0
With non-negative weights and increasing activations y is non-decreasing in
every feature, and every feature is non-decreasing in the code, so y is
non-decreasing in the key.
"""
from __future__ import annotations

import numpy as np

H = 64
NF = 8
PARAM_SHAPES = {"W1": (H, NF), "b1": (H,), "W2": (H, H), "b2": (H,), "w3": (H,), "b3": (1,)}
NONNEG = ("W1", "W2", "w3")
N_PARAMS = sum(int(np.prod(s)) for s in PARAM_SHAPES.values())  # 4801


def knots(sorted_codes: np.ndarray):
    """q_0..q_8 (codes at the 1/8 quantiles and the largest) and widths w_0..w_7."""
    c = np.asarray(sorted_codes, dtype=np.uint64)
    S = c.size
    q = np.array([c[(k * S) // 8] for k in range(8)] + [c[S - 1]], dtype=np.uint64)
    w = np.maximum(q[1:].astype(np.float64) - q[:-1].astype(np.float64), 1.0)
    return q, w


def features(codes: np.ndarray, q: np.ndarray, w: np.ndarray) -> np.ndarray:
    c = np.asarray(codes, dtype=np.uint64)
    d = np.where(c[:, None] >= q[None, :8], c[:, None] - q[None, :8], np.uint64(0)).astype(np.float64)
    return np.minimum(d / w[None, :], 1.0)


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(P: dict, X: np.ndarray, bf16_layer2: bool = False):
    """Intermediates and output for a batch of feature rows X (n x 8)."""
    z1 = X @ P["W1"].T + P["b1"]
    h1 = sigmoid(z1)
    h1q = bf16(h1) if bf16_layer2 else h1
    W2 = bf16(P["W2"]) if bf16_layer2 else P["W2"]
    z2 = h1q @ W2.T + P["b2"]
    h2 = sigmoid(z2)
    y = h2 @ P["w3"] + P["b3"][0]
    return {"z1": z1, "h1": h1, "h1q": h1q, "W2q": W2, "z2": z2, "h2": h2, "y": y}


def loss_and_grads(P: dict, X: np.ndarray, t: np.ndarray, bf16_layer2: bool = False, bf16_dz2: bool = False):
    """Mean squared error to the targets t and its gradient w.r.t. every parameter.
    ``bf16_dz2`` rounds dL/dz2 to bfloat16 where it enters the two 64x64
    products of the backward pass (dW2 and dh1), as the GPU's matrix cores take it."""
    f = forward(P, X, bf16_layer2)
    M = X.shape[0]
    r = f["y"] - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / M
    g = {"w3": f["h2"].T @ dy, "b3": np.array([dy.sum()])}
    dz2 = np.outer(dy, P["w3"]) * f["h2"] * (1.0 - f["h2"])
    dz2q = bf16(dz2) if bf16_dz2 else dz2
    g["W2"] = dz2q.T @ f["h1q"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2q @ f["W2q"]
    dz1 = dh1 * f["h1"] * (1.0 - f["h1"])
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return loss, g


def initial_params(u: np.ndarray) -> dict:
    """Starting point from N_PARAMS uniform draws u in [0, 1), in the flat
    parameter order: W1 ~ U(0, 1), b1 ~ U(-4, 0), W2 ~ U(0, 0.1), b2 = -3,
    w3 ~ U(0, 0.05), b3 = 0 -- small positive weights, units off saturation."""
    P = unpack(np.asarray(u, dtype=np.float64))
    P["b1"] = -4.0 * P["b1"]
    P["W2"] = 0.1 * P["W2"]
    P["b2"] = np.full(H, -3.0)
    P["w3"] = 0.05 * P["w3"]
    P["b3"] = np.zeros(1)
    return P


def adam_step(P: dict, m: dict, v: dict, g: dict, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1), then W1, W2, w3 projected to >= 0."""
    for k in P:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
        if k in NONNEG:
            P[k] = np.maximum(P[k], 0.0)


def unpack(flat: np.ndarray) -> dict:
    """Parameters from the flat layout W1, b1, W2, b2, w3, b3 (row-major)."""
    P, o = {}, 0
    for k, s in PARAM_SHAPES.items():
        n = int(np.prod(s))
        P[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(s).copy()
        o += n
    return P


def pack(P: dict) -> np.ndarray:
    return np.concatenate([np.asarray(P[k], dtype=np.float64).ravel() for k in PARAM_SHAPES])


def _after_run(c: np.ndarray, q: np.ndarray) -> np.ndarray:
    """Leaves whose start sample q[j] lies in the same run of equal codes as
    the previous leaf's start sample."""
    a = np.zeros(q.size, dtype=bool)
    a[1:] = c[q[1:]] == c[q[:-1]]
    return a


def equi_depth_first(sorted_codes: np.ndarray, L: int) -> np.ndarray:
    """Leaf ranges under the equi-depth roots (MLP and spline): leaf j starts
    at the first sample of the run of equal codes that holds sample
    floor(j*S/L), so a run of equal keys is never split between leaves --
    except that a run holding the start samples of several leaves becomes a
    leaf of its own: the first of those leaves covers exactly the run, and the
    others start after it (the run's code then has a bucket to itself, whose
    keys are all equal).  first[L] = S."""
    c = np.asarray(sorted_codes, dtype=np.uint64)
    S = c.size
    q = (np.arange(L, dtype=np.int64) * S) // L
    first = np.searchsorted(c, c[q], side="left")
    after = _after_run(c, q)
    first[after] = np.searchsorted(c, c[q[after]], side="right")
    return np.append(first, S).astype(np.uint64)


def equi_depth_bound(sorted_codes: np.ndarray, L: int) -> np.ndarray:
    """Routing boundaries of those leaves (leaf j takes the codes in
    [bound[j], bound[j+1])): 0 for leaf 0; the code of the leaf's first sample;
    for a leaf that starts after a run of code v, v + 1 (so the run's own leaf
    holds that one code); past every code for a leaf with no samples after
    it, and for bound[L]."""
    c = np.asarray(sorted_codes, dtype=np.uint64)
    S = c.size
    first = equi_depth_first(c, L).astype(np.int64)
    q = (np.arange(L, dtype=np.int64) * S) // L
    after = _after_run(c, q)
    top = np.iinfo(np.uint64).max
    bound = np.full(L + 1, top, dtype=np.uint64)
    for j in range(1, L):
        if after[j]:
            bound[j] = c[q[j]] + np.uint64(1)
        elif first[j] < S:
            bound[j] = c[first[j]]
    bound[0] = 0
    return bound


def leaf_guess(y: np.ndarray, L: int) -> np.ndarray:
    """The router's starting leaf floor(L*y), clamped to [0, L-1]."""
    return np.clip(np.floor(np.asarray(y) * L), 0, L - 1).astype(np.int64)
