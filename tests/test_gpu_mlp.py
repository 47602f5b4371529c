"""The predictor network's HIP kernels (binary32) against the FP64 reference:
outputs, loss, every gradient tensor, Adam, and a short fit."""
import numpy as np
import pytest

import matgen
from oracle import mlp as ref
from paper_2204_06666_amd.predictor import N_PARAMS, SHAPES, Mlp, init_params

pytestmark = pytest.mark.gpu

import torch  # noqa: E402


def _data(b, seed):
    g = matgen.rng(seed)
    return g.normal(size=(b, 32)).astype(np.float32), g.normal(size=(b, 3)).astype(np.float32)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("batch", [1, 7, 64, 1000, 5000])
def test_forward_and_gradients(batch):
    p = init_params(batch)
    p[ref.N_PARAMS - 3:] = [0.1, -0.2, 0.3]
    X, T = _data(batch, batch + 1)
    net = Mlp(p)
    Y = net.forward(_dev(X)).cpu().numpy()
    y64, _ = ref.forward(p.astype(np.float64), X.astype(np.float64))
    assert _rel(Y, y64) <= 1e-5
    g, L = net.grad(_dev(X), _dev(T))
    L64, g64 = ref.grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert abs(L.item() - L64) <= 1e-5 * L64
    g, o = g.cpu().numpy().astype(np.float64), 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        err = _rel(g[o:o + k], g64[o:o + k])
        assert err <= 1e-4, (name, batch, err)
        o += k
    print(f"[mlp] batch={batch} loss={L.item():.6f} vs {L64:.6f}", flush=True)


def test_gradients_reproducible():
    X, T = _data(3000, 5)
    net = Mlp(init_params(3))
    g0 = net.grad(_dev(X), _dev(T))[0].clone()
    for _ in range(3):
        assert torch.equal(net.grad(_dev(X), _dev(T))[0], g0)


def test_adam_steps_match_reference():
    p = init_params(9).astype(np.float64)
    X, T = _data(200, 10)
    net = Mlp(p)
    m = np.zeros(N_PARAMS)
    v = np.zeros(N_PARAMS)
    for step in range(1, 4):
        net.grad(_dev(X), _dev(T))
        g = net.grad_buf.cpu().numpy().astype(np.float64)
        net.adam(1e-3)
        p, m, v = ref.adam(p, g, m, v, step, 1e-3)
        assert np.allclose(net.numpy_params(), p, rtol=1e-5, atol=1e-6), step


def test_fit_learns_a_teacher():
    """Targets from a random teacher network: the loss falls by 10x."""
    X, _ = _data(4096, 20)
    teacher = init_params(21).astype(np.float64)
    T, _ = ref.forward(teacher, X.astype(np.float64))
    T = (T / np.abs(T).max()).astype(np.float32)
    net = Mlp(seed=22)
    hist = net.fit(_dev(X), _dev(T), epochs=30, batch=256, lr=3e-3, seed=1)
    print(f"[mlp] fit loss {hist[0]:.4e} -> {hist[-1]:.4e}", flush=True)
    assert hist[-1] < 0.1 * hist[0]
    assert ref.loss(net.numpy_params().astype(np.float64), X, T) < 0.1 * hist[0]
