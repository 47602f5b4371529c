"""Pins of the FP64 reference network: gradients against central finite
differences, and cases with closed-form results."""
import numpy as np

import matgen
from oracle import mlp


def _params(seed, scale=1.0):
    g = matgen.rng(seed)
    d = {}
    for name, shape in mlp.SHAPES:
        fan_in = shape[1] if len(shape) == 2 else 1
        d[name] = g.normal(0, scale * np.sqrt(2.0 / fan_in), shape) if len(shape) == 2 else g.normal(0, 0.1, shape)
    return mlp.pack(d)


def test_gradient_matches_central_differences():
    g = matgen.rng(1)
    p = _params(2)
    X = g.normal(size=(7, 32))
    T = g.normal(size=(7, 3))
    _, gr = mlp.grad(p, X, T)
    h = 1e-6
    idx = np.concatenate([g.choice(mlp.N_PARAMS, 300, replace=False), np.arange(mlp.N_PARAMS - 3, mlp.N_PARAMS)])
    fd = np.empty(idx.size)
    for k, i in enumerate(idx):
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd[k] = (mlp.loss(p + e, X, T) - mlp.loss(p - e, X, T)) / (2 * h)
    err = np.linalg.norm(fd - gr[idx]) / np.linalg.norm(gr[idx])
    assert err <= 1e-6, err


def test_closed_forms():
    """Zero weights: y = b3, so dL/db3 = 2 mean_b (b3 - t) / 3 and every
    other gradient is 0.  A one-hidden-path network computes a known value."""
    g = matgen.rng(3)
    X = g.normal(size=(5, 32))
    T = g.normal(size=(5, 3))
    p = np.zeros(mlp.N_PARAMS)
    w = mlp.unpack(p)
    w["b3"] = np.array([0.5, -1.0, 2.0])
    p = mlp.pack(w)
    L, gr = mlp.grad(p, X, T)
    assert np.isclose(L, np.mean((w["b3"] - T) ** 2))
    gw = mlp.unpack(gr)
    assert np.allclose(gw["b3"], 2 * np.mean(w["b3"] - T, axis=0) / 3)
    assert all(np.all(gw[k] == 0) for k in ("W1", "b1", "W2", "b2", "W3"))
    # y_0 = relu(relu(x_0) * 2) * 3 for W1[0,0] = 1, W2[0,0] = 2, W3[0,0] = 3
    w = {k: np.zeros(s) for k, s in mlp.SHAPES}
    w["W1"][0, 0], w["W2"][0, 0], w["W3"][0, 0] = 1.0, 2.0, 3.0
    X = np.zeros((3, 32))
    X[:, 0] = [-1.0, 0.5, 2.0]
    y, _ = mlp.forward(mlp.pack(w), X)
    assert np.array_equal(y[:, 0], [0.0, 3.0, 12.0]) and np.all(y[:, 1:] == 0)


def test_adam_first_step_is_signed_lr():
    """After one step from zero moments, the bias-corrected update is
    lr * g / (|g| + eps): every parameter moves by about lr against its gradient."""
    g = matgen.rng(4).normal(size=mlp.N_PARAMS)
    p = np.zeros(mlp.N_PARAMS)
    p1, m, v = mlp.adam(p, g, np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    assert np.allclose(p1, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
