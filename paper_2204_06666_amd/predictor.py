"""Learned preprocessing parameters: the network of ehyb_mlp_* (forward,
gradient and Adam all run in the library's own HIP kernels) and the mapping
between its three outputs and the grid of (partition size, ELL width cap,
rows per wave).

The paper sizes partitions by a fixed rule (Eq. 1) and has no ELL width or
lane-count parameter; these are tuned per matrix here, by an exhaustive sweep
(``autotune``) whose best points train the network.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import check, load

N_IN, N_HID, N_OUT, N_PARAMS = 32, 64, 3, 6467
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]

# the tuning grid (FP32 values, one right-hand side).  Partition sizes reach
# down to 256 rows so that matrices of 10^4 - 10^5 rows can still spread over
# the 256 CUs; 0 is the LDS limit ((160 KiB - 64) / 8 rows).
SLICE_ROWS = (256, 512, 1024, 2048, 4096, 0)
WIDTH_QUANTILES = (None, 0.99, 0.90, 0.75)        # ELL width cap: the library's automatic cap or a row-length quantile
ROWS_PER_WAVE = (8, 16, 32, 64)


def lds_max_rows(x_bytes: int = 4, n_rhs: int = 1, lds: int = 160 * 1024) -> int:
    return min(65535, (lds - 64) // (2 * x_bytes * n_rhs))


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, float32."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _, shape in SHAPES:
        parts.append(g.normal(0.0, np.sqrt(2.0 / shape[1]), shape).reshape(-1) if len(shape) == 2
                     else np.zeros(shape[0]))
    return np.concatenate(parts).astype(np.float32)


class Mlp:
    """Parameters and Adam moments on the device; every step is a library call."""

    def __init__(self, params=None, seed: int = 0, device="cuda:0"):
        import torch
        self._lib = load()
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float32)
        if p.shape != (N_PARAMS,):
            raise ValueError(f"expected {N_PARAMS} parameters")
        self.device = torch.device(device)
        self.params = torch.from_numpy(p.copy()).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad_buf = torch.zeros_like(self.params)
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=self.device)
        self.step = 0
        self._ws = None

    def _check_x(self, X, cols):
        import torch
        if X.dtype != torch.float32 or not X.is_cuda or not X.is_contiguous() or X.dim() != 2 or X.shape[1] != cols:
            raise ValueError(f"expected a contiguous float32 CUDA tensor [batch, {cols}]")

    def forward(self, X, Y=None, stream=None):
        import torch
        self._check_x(X, N_IN)
        Y = torch.empty(X.shape[0], N_OUT, dtype=torch.float32, device=X.device) if Y is None else Y
        check(self._lib.ehyb_mlp_forward(_ptr(self.params), X.shape[0], _ptr(X), _ptr(Y), _stream(stream)),
              "ehyb_mlp_forward")
        return Y

    def grad(self, X, T, stream=None):
        """Fills self.grad_buf and self.loss_buf; returns them."""
        import torch
        self._check_x(X, N_IN)
        self._check_x(T, N_OUT)
        b = X.shape[0]
        need = ctypes.c_size_t()
        check(self._lib.ehyb_mlp_workspace_bytes(b, ctypes.byref(need)), "ehyb_mlp_workspace_bytes")
        if self._ws is None or self._ws.numel() < need.value:
            self._ws = torch.empty(need.value, dtype=torch.uint8, device=self.device)
        check(self._lib.ehyb_mlp_grad(_ptr(self.params), b, _ptr(X), _ptr(T), _ptr(self.grad_buf),
                                      _ptr(self.loss_buf), _ptr(self._ws), self._ws.numel(), _stream(stream)),
              "ehyb_mlp_grad")
        return self.grad_buf, self.loss_buf

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, stream=None):
        self.step += 1
        check(self._lib.ehyb_mlp_adam(_ptr(self.params), _ptr(self.grad_buf), _ptr(self.m), _ptr(self.v),
                                      self.step, lr, beta1, beta2, eps, _stream(stream)), "ehyb_mlp_adam")

    def fit(self, X, T, epochs: int, batch: int, lr: float, seed: int = 0):
        """Minibatch Adam on device tensors X [n, 32], T [n, 3]; the order of
        the samples is reshuffled every epoch (seeded).  Returns the mean
        minibatch loss of every epoch."""
        import torch
        n = X.shape[0]
        g = np.random.Generator(np.random.PCG64(seed))
        hist = []
        for _ in range(epochs):
            order = torch.from_numpy(g.permutation(n)).to(X.device)
            Xs, Ts = X[order].contiguous(), T[order].contiguous()
            tot = torch.zeros(1, dtype=torch.float32, device=X.device)
            k = 0
            for s in range(0, n, batch):
                self.grad(Xs[s:s + batch], Ts[s:s + batch])
                self.adam(lr)
                tot += self.loss_buf
                k += 1
            hist.append(float(tot.item()) / k)
        return hist

    def numpy_params(self) -> np.ndarray:
        return self.params.cpu().numpy().copy()


# ---------------------------------------------------------------- targets
def encode_target(slice_rows: int, width_q, rows_per_wave: int) -> np.ndarray:
    """Grid point -> three network targets: index of the partition size,
    index of the width cap and log2(rows_per_wave) - 3, each scaled to [0, 1]."""
    return np.array([SLICE_ROWS.index(slice_rows) / (len(SLICE_ROWS) - 1),
                     WIDTH_QUANTILES.index(width_q) / (len(WIDTH_QUANTILES) - 1),
                     (np.log2(rows_per_wave) - 3) / 3.0], dtype=np.float32)


def decode_output(y: np.ndarray):
    """Network output -> nearest grid point (slice_rows, width quantile, rows_per_wave)."""
    i = int(np.clip(np.rint(y[0] * (len(SLICE_ROWS) - 1)), 0, len(SLICE_ROWS) - 1))
    j = int(np.clip(np.rint(y[1] * (len(WIDTH_QUANTILES) - 1)), 0, len(WIDTH_QUANTILES) - 1))
    k = int(np.clip(np.rint(y[2] * 3.0), 0, 3))
    return SLICE_ROWS[i], WIDTH_QUANTILES[j], ROWS_PER_WAVE[k]


def width_cap(row_lengths: np.ndarray, q) -> int:
    """ELL width cap of quantile q (lower quantile of the row lengths, at least 1);
    None gives 0, the library's automatic cap."""
    if q is None:
        return 0
    s = np.sort(np.asarray(row_lengths))
    return max(1, int(s[int(np.floor(q * (s.size - 1)))])) if s.size else 0
