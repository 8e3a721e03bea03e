"""FP64 NumPy oracle of the small proposal network (4 -> 64 -> 64 -> 1, tanh,
tanh, logistic output, mean squared error, Adam).

TEST INFRASTRUCTURE ONLY: used by the tests to check the GPU forward,
backward and Adam kernels; shares no code with them.  Parameters use the same
flat layout as the GPU library: W1[64][4] b1[64] W2[64][64] b2[64] W3[64] b3.
Backpropagation is written out layer by layer (chain rule), with no
framework.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID = 4, 64
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("W3", (N_HID,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def forward(p, X):
    """Returns (out (B,), h1 (B,64), h2 (B,64))."""
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ w["W1"].T + w["b1"])
    h2 = np.tanh(h1 @ w["W2"].T + w["b2"])
    z3 = h2 @ w["W3"] + w["b3"][0]
    out = 1.0 / (1.0 + np.exp(-z3))
    return out, h1, h2


def loss(p, X, Y):
    out, _, _ = forward(p, X)
    return float(np.mean((out - np.asarray(Y, dtype=np.float64)) ** 2))


def backward(p, X, Y):
    """Gradient of the mean squared error with respect to the flat parameters."""
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    B = X.shape[0]
    out, h1, h2 = forward(p, X)
    d3 = 2.0 / B * (out - Y) * out * (1.0 - out)          # dL/dz3
    d2 = np.outer(d3, w["W3"]) * (1.0 - h2 ** 2)           # dL/dz2
    d1 = (d2 @ w["W2"]) * (1.0 - h1 ** 2)                  # dL/dz1
    g = {"W3": d3 @ h2, "b3": np.array([d3.sum()]), "W2": d2.T @ h1, "b2": d2.sum(0),
         "W1": d1.T @ X, "b1": d1.sum(0)}
    return np.concatenate([g[name].ravel() for name, _ in SIZES])


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, bias-corrected).  Returns (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """Glorot-uniform weights, zero biases (same recipe the GPU driver uses)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SIZES:
        if name.startswith("W"):
            fan_in = shape[-1] if len(shape) > 1 else N_HID
            fan_out = shape[0] if len(shape) > 1 else 1
            lim = np.sqrt(6.0 / (fan_in + fan_out))
            parts.append(rng.uniform(-lim, lim, size=shape).ravel())
        else:
            parts.append(np.zeros(shape).ravel())
    return np.concatenate(parts)
