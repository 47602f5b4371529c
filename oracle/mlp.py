"""Reference of the parameter-predictor network (test infrastructure only).

A fully connected network in FP64, written out layer by layer:
    z1 = W1 x + b1, h1 = relu(z1), z2 = W2 h1 + b2, h2 = relu(z2), y = W3 h2 + b3,
with x of 32 features, two hidden layers of 64 units and 3 outputs; loss
L = sum over samples b and outputs o of (y_bo - t_bo)^2 / (B * 3) and its
gradient by the chain rule (relu'(0) = 0).  Parameters are one flat vector:
W1 [64][32] row-major, b1 [64], W2 [64][64], b2 [64], W3 [3][64], b3 [3].
Adam follows Kingma and Ba (2015), Algorithm 1.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 32, 64, 3
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def forward(p: np.ndarray, X: np.ndarray):
    """Outputs [B][3] and the intermediate values of every layer."""
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["W3"].T + w["b3"]
    return y, (X, z1, h1, z2, h2)


def loss(p: np.ndarray, X: np.ndarray, T: np.ndarray) -> float:
    y, _ = forward(p, X)
    return float(np.sum((y - T) ** 2) / y.size)


def grad(p: np.ndarray, X: np.ndarray, T: np.ndarray):
    """(loss, dL/dp) by backpropagation."""
    w = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    dy = 2.0 * (y - T) / y.size
    g = {"W3": dy.T @ h2, "b3": dy.sum(axis=0)}
    dz2 = (dy @ w["W3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ w["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return float(np.sum((y - T) ** 2) / y.size), pack(g)


def adam(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
