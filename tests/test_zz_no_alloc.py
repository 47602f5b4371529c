"""ehyb_mlp_grad_noalloc (the gradient with the library's static scratch in
place of the caller's workspace) against ehyb_mlp_grad, through the C ABI:
the same bits on two calls in a row, the second with a smaller batch (the
scratch keeps the first call's partial sums), and the FP64 reference network
within the binary32 bound the gradient tests use."""
import ctypes

import numpy as np
import pytest

import matgen
from oracle import mlp as ref
from paper_2204_06666_amd import _abi
from paper_2204_06666_amd.predictor import N_PARAMS, init_params

pytestmark = pytest.mark.gpu

import torch  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _with_workspace(lib, p, X, T):
    batch = X.shape[0]
    need = ctypes.c_size_t(0)
    assert lib.ehyb_mlp_workspace_bytes(batch, ctypes.byref(need)) == _abi.EHYB_OK
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda:0")
    g = torch.empty(N_PARAMS, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    st = lib.ehyb_mlp_grad(_ptr(p), batch, _ptr(X), _ptr(T), _ptr(g), _ptr(loss), _ptr(ws), need.value, _stream())
    assert st == _abi.EHYB_OK, lib.ehyb_last_error()
    return g, loss


def _without_allocation(lib, p, X, T):
    g = torch.empty(N_PARAMS, dtype=torch.float32, device="cuda:0")
    loss = torch.empty(1, dtype=torch.float32, device="cuda:0")
    st = lib.ehyb_mlp_grad_noalloc(_ptr(p), X.shape[0], _ptr(X), _ptr(T), _ptr(g), _ptr(loss), _stream())
    assert st == _abi.EHYB_OK, lib.ehyb_last_error()
    return g, loss


def test_noalloc_gradient_equals_workspace_gradient_on_two_calls():
    lib = _abi.load()
    p32 = init_params(5)
    p = _dev(p32)
    # the largest grid first (256 workgroups), then a smaller batch (10 of them)
    for batch, seed in ((3000, 21), (37, 22)):
        g = matgen.rng(seed)
        X32 = g.normal(size=(batch, 32)).astype(np.float32)
        T32 = g.normal(size=(batch, 3)).astype(np.float32)
        X, T = _dev(X32), _dev(T32)
        g_ws, l_ws = _with_workspace(lib, p, X, T)
        g_na, l_na = _without_allocation(lib, p, X, T)
        torch.cuda.synchronize()
        print(f"[noalloc] batch={batch} loss={l_na.item():.6g}", flush=True)
        assert torch.equal(g_na.view(torch.int32), g_ws.view(torch.int32)), f"batch {batch}: gradients differ"
        assert torch.equal(l_na.view(torch.int32), l_ws.view(torch.int32)), f"batch {batch}: losses differ"
        L64, g64 = ref.grad(p32.astype(np.float64), X32.astype(np.float64), T32.astype(np.float64))
        gn = g_na.cpu().numpy().astype(np.float64)
        assert np.linalg.norm(gn - g64) <= 1e-4 * np.linalg.norm(g64)
        assert abs(l_na.item() - L64) <= 1e-5 * L64


def test_noalloc_rejects_bad_arguments():
    lib = _abi.load()
    z = ctypes.c_void_p(0)
    assert lib.ehyb_mlp_grad_noalloc(z, 0, z, z, z, z, z) == _abi.EHYB_EINVAL
    assert lib.ehyb_mlp_grad_noalloc(z, 4, z, z, z, z, z) == _abi.EHYB_EINVAL
