"""CPU float64 reference of the work-predictor MLP -- TEST INFRASTRUCTURE ONLY.

Network: 4 -> 64 -> 64 -> 1 with ReLU after both hidden layers,
y = W3 relu(W2 relu(W1 x + b1) + b2) + b3, loss = mean((y - t)^2), and the
Adam update of Kingma and Ba (2015) with beta1 = 0.9, beta2 = 0.999,
eps = 1e-8.  Parameter block layout (flat, row-major):
W1[64][4] b1[64] W2[64][64] b2[64] W3[64] b3[1].

Only the tests may import this module.  Pinned in tests/test_mlp_oracle.py by
hand-computed outputs, central finite differences of the loss (for the
gradient) and the closed form of Adam's first step.
"""
from __future__ import annotations

import numpy as np

NIN, H = 4, 64
SIZES = [("W1", (H, NIN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, x):
    P = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    return h2 @ P["W3"] + P["b3"][0]


def loss(p, x, t):
    y = forward(p, x)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def loss_and_grad(p, x, t):
    """Mean squared error and its gradient by the chain rule."""
    P = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B = x.shape[0]
    z1 = x @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["W3"] + P["b3"][0]
    err = y - t
    dy = 2.0 * err / B
    g = {}
    g["W3"] = dy @ h2
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, P["W3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ x
    g["b1"] = dz1.sum(axis=0)
    return float(np.mean(err ** 2)), pack(g)


def grad_magnitude(p, x, t):
    """The magnitude each gradient entry is computed from: the chain rule of
    loss_and_grad with every weight, input, target and intermediate replaced
    by its absolute value (ReLU masks kept).  Rounding in any order of the
    same products and sums moves an entry by at most a small multiple of
    (number of rounded operations) x unit roundoff x this magnitude, the
    classical forward error bound for sums and dot products."""
    P = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B = x.shape[0]
    z1 = x @ P["W1"].T + P["b1"]
    m1 = z1 > 0
    z2 = np.maximum(z1, 0.0) @ P["W2"].T + P["b2"]
    m2 = z2 > 0
    a1 = (np.abs(x) @ np.abs(P["W1"]).T + np.abs(P["b1"])) * m1
    a2 = (a1 @ np.abs(P["W2"]).T + np.abs(P["b2"])) * m2
    ya = a2 @ np.abs(P["W3"]) + abs(P["b3"][0])
    dya = 2.0 * (ya + np.abs(t)) / B
    dz2a = np.outer(dya, np.abs(P["W3"])) * m2
    dz1a = (dz2a @ np.abs(P["W2"])) * m1
    g = {"W3": dya @ a2, "b3": np.array([dya.sum()]), "W2": dz2a.T @ a1, "b2": dz2a.sum(axis=0),
         "W1": dz1a.T @ np.abs(x), "b1": dz1a.sum(axis=0)}
    return pack(g)


def relu_margin(p, x):
    """Per row: the smallest |pre-activation| of either hidden layer relative
    to the magnitude of its terms.  Rows with a tiny margin may have a ReLU
    mask that rounding can flip."""
    P = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ P["W1"].T + P["b1"]
    a1 = np.abs(x) @ np.abs(P["W1"]).T + np.abs(P["b1"])
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    a2 = h1 @ np.abs(P["W2"]).T + np.abs(P["b2"])
    r1 = np.abs(z1) / np.maximum(a1, 1e-300)
    r2 = np.abs(z2) / np.maximum(a2, 1e-300)
    return np.minimum(r1.min(axis=1), r2.min(axis=1))


def adam_step(p, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-style initialisation (normal, std sqrt(2 / fan_in)), zero biases."""
    r = np.random.default_rng(seed)
    d = {
        "W1": r.normal(0, np.sqrt(2.0 / NIN), (H, NIN)), "b1": np.zeros(H),
        "W2": r.normal(0, np.sqrt(2.0 / H), (H, H)), "b2": np.zeros(H),
        "W3": r.normal(0, np.sqrt(1.0 / H), (H,)), "b3": np.zeros(1),
    }
    return pack(d)
