"""FP64 CPU twin of the pruner MLP (42 -> 128 -> 128 -> 128 -> 1, ReLU, sigmoid).

TEST INFRASTRUCTURE: used to check the GPU forward / backward kernels.  Plain
numpy, float64.  Parameter layout (flat vector of 38657 values): W1 [42 x 128]
(row = input), b1 [128], W2 [128 x 128], b2, W3 [128 x 128], b3, W4 [128], b4 [1].
Loss: mean over the batch of  -w y log p - (1 - y) log(1 - p),  w = pos_weight
for positives, p = sigmoid(z).
"""
from __future__ import annotations

import numpy as np

IN, HID = 42, 128
SIZES = [("W1", (IN, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (HID, HID)),
         ("b3", (HID,)), ("W4", (HID,)), ("b4", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def features(P, N, tri, x0s, x3s, q_x0, q_x3, q_tris) -> np.ndarray:
    """[n, 42]: x0/2, x3/2, positions of T1 and T2 / 2, normals of T1 and T2."""
    t1, t2 = q_tris[:, 0], q_tris[:, 1]
    f = [x0s[q_x0] * 0.5, x3s[q_x3] * 0.5]
    f += [P[tri[t1, v]] * 0.5 for v in range(3)]
    f += [P[tri[t2, v]] * 0.5 for v in range(3)]
    f += [N[tri[t1, v]] for v in range(3)]
    f += [N[tri[t2, v]] for v in range(3)]
    return np.concatenate(f, axis=1)


def forward(p: np.ndarray, X: np.ndarray):
    W = unpack(p)
    z1 = X @ W["W1"] + W["b1"]
    h1 = np.maximum(z1, 0)
    z2 = h1 @ W["W2"] + W["b2"]
    h2 = np.maximum(z2, 0)
    z3 = h2 @ W["W3"] + W["b3"]
    h3 = np.maximum(z3, 0)
    z4 = h3 @ W["W4"] + W["b4"][0]
    return z4, (z1, h1, z2, h2, z3, h3)


def loss_and_grad(p: np.ndarray, X: np.ndarray, y: np.ndarray, pos_w: float):
    W = unpack(p)
    z4, (z1, h1, z2, h2, z3, h3) = forward(p, X)
    n = len(y)
    sp_neg = np.logaddexp(0.0, -z4)      # -log sigmoid(z)
    sp_pos = np.logaddexp(0.0, z4)       # -log(1 - sigmoid(z))
    w = np.where(y > 0.5, pos_w, 1.0)
    loss = np.sum(w * y * sp_neg + (1 - y) * sp_pos) / n
    pr = 1.0 / (1.0 + np.exp(-z4))
    g4 = (w * y * (pr - 1.0) + (1 - y) * pr) / n
    G = {}
    G["W4"] = h3.T @ g4
    G["b4"] = np.array([g4.sum()])
    d3 = np.outer(g4, W["W4"]) * (z3 > 0)
    G["W3"] = h2.T @ d3
    G["b3"] = d3.sum(0)
    d2 = (d3 @ W["W3"].T) * (z2 > 0)
    G["W2"] = h1.T @ d2
    G["b2"] = d2.sum(0)
    d1 = (d2 @ W["W2"].T) * (z1 > 0)
    G["W1"] = X.T @ d1
    G["b1"] = d1.sum(0)
    g = np.concatenate([G[name].ravel() for name, _ in SIZES])
    return loss, g


def init_params(seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SIZES:
        if name.startswith("W"):
            fan_in = shape[0]
            lim = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, shape).ravel())
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts)
