"""Oracle of the selector network's training arithmetic (test infrastructure only).

Network 16 -> 32 -> 32 -> 3 with ReLU; parameters flat in the order W1[32][16],
b1[32], W2[32][32], b2[32], W3[3][32], b3[3].  Training loss: softmax
cross-entropy of the logits against the exhaustive trial's label, averaged
over the batch; optimiser: Adam (Kingma and Ba, 2015) with bias correction.
Everything here is float64 and follows the textbook definitions; the pins
check the gradient by central finite differences.
"""
from __future__ import annotations

import numpy as np

NPARAM = 1699
SHAPES = (("W1", (32, 16)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (3, 32)), ("b3", (3,)))


def unpack(w):
    w = np.asarray(w, np.float64)
    out, o = {}, 0
    for name, shp in SHAPES:
        size = int(np.prod(shp))
        out[name] = w[o:o + size].reshape(shp)
        o += size
    assert o == NPARAM
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], np.float64).reshape(-1) for name, _ in SHAPES])


def forward(w, x):
    p = unpack(w)
    x = np.asarray(x, np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["W3"].T + p["b3"]
    return z1, h1, z2, h2, z3


def loss(w, x, y):
    z3 = forward(w, x)[4]
    m = z3.max(axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(z3 - m).sum(axis=1))
    return float(np.mean(lse - z3[np.arange(len(y)), y]))


def grad(w, x, y):
    """Gradient of the mean cross-entropy with respect to the flat parameters."""
    p = unpack(w)
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.int64)
    B = x.shape[0]
    z1, h1, z2, h2, z3 = forward(w, x)
    e = np.exp(z3 - z3.max(axis=1, keepdims=True))
    sm = e / e.sum(axis=1, keepdims=True)
    dz3 = sm.copy()
    dz3[np.arange(B), y] -= 1.0
    dz3 /= B
    dh2 = dz3 @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    return pack({"W1": dz1.T @ x, "b1": dz1.sum(0), "W2": dz2.T @ h1, "b2": dz2.sum(0),
                 "W3": dz3.T @ h2, "b3": dz3.sum(0)})


def adam(w, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
