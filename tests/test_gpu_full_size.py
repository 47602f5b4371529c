"""Full-size parity of the benchmarked unstructured-FEM and batched workloads,
in the launch configurations the benchmark times, every row against the oracle.

* Mutual-kNN FEM stand-in: 10^6 points ~ U[0,1]^3, 3x3 blocks, 3e6 rows and
  1.94e8 nnz.  Default plan parameters and the automatic load mode, which
  gives streaming loads at this size.  FP64 must agree within
  1e-12 * sum |a x| per row.  FP32, BF16 and their binary64-accumulating
  variants must agree with the FP64 product of the stored values within the
  accumulation bound (Higham's gamma_m of the unit roundoff the sums use).
* 64 uneven matrices x 8 right-hand sides, FP32, with the tuned plan
  parameters.  One launch is recorded in a HIP graph and replayed; the
  replay must equal an eager launch bit for bit, and every row must lie
  within the binary32 accumulation bound.
"""
import numpy as np
import pytest

import matgen
import oracle
from oracle.precision import gamma32, quantize
from paper_2204_06666_amd import (EHYB_BF16, EHYB_BF16_ACC64, EHYB_F32, EHYB_F32_ACC64, EHYB_F64, Batch,
                                  Plan)
from paper_2204_06666_amd.workloads import BATCHED_PARAMS, batched_tuned

pytestmark = pytest.mark.gpu

import torch  # noqa: E402


def _gamma64(m):
    u = 2.0 ** -53
    return m * u / (1.0 - m * u)


@pytest.fixture(scope="module")
def knn():
    print("[full-size] generating the kNN-FEM matrix (1e6 points)", flush=True)
    A = matgen.config_matrix(3)
    x = matgen.uniform_vector(A.n_rows, matgen.CONFIG_SEEDS[3] + 2)
    assert A.n_rows == 3_000_000
    return A, x


def _product(A, x, dt):
    P = Plan(A, value_dtype=dt).upload("cuda:0")
    perm = P.perm()
    xt = torch.from_numpy(x[perm].astype(np.float64 if dt == EHYB_F64 else np.float32)).to("cuda:0")
    yt = torch.empty_like(xt)
    P.spmv(xt, yt)
    torch.cuda.synchronize()
    y = np.empty(A.n_rows)
    y[perm] = yt.cpu().numpy()
    del P, xt, yt
    torch.cuda.empty_cache()
    return y


@pytest.mark.timeout(900)
def test_knn_fem_full_size_fp64(knn):
    A, x = knn
    print(f"[full-size] kNN-FEM FP64 n={A.n_rows} nnz={A.nnz}", flush=True)
    w = oracle.assert_close(_product(A, x, EHYB_F64), oracle.spmv(A, x), oracle.abs_scale(A, x), 1e-12,
                            "kNN-FEM FP64")
    print(f"[full-size] kNN-FEM FP64 worst scaled error {w:.2e}", flush=True)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dt", [EHYB_F32, EHYB_BF16, EHYB_F32_ACC64, EHYB_BF16_ACC64])
def test_knn_fem_full_size_low_precision(knn, dt):
    A, x = knn
    kind = "bf16" if dt in (EHYB_BF16, EHYB_BF16_ACC64) else "f32"
    print(f"[full-size] kNN-FEM value type {dt} ({kind})", flush=True)
    y = _product(A, x, dt)
    Aq = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, quantize(A.val, kind))
    xq = x.astype(np.float32).astype(np.float64)
    yq = oracle.spmv(Aq, xq)
    sq = oracle.abs_scale(Aq, xq)
    m = np.diff(A.row_ptr).astype(np.float64)
    if dt in (EHYB_F32_ACC64, EHYB_BF16_ACC64):
        bound = (2.0 ** -24 + _gamma64(m + 2) * (1 + 2.0 ** -24)) * sq
    else:
        bound = gamma32(m + 2) * sq
    err = np.abs(y - yq)
    bad = ~((err <= bound) | ((sq == 0) & (y == yq)))
    assert not bad.any(), f"value type {dt}: {bad.sum()} rows outside the bound, first {np.argmax(bad)}"
    print(f"[full-size] value type {dt}: worst error / sum|a x| "
          f"{np.max(err / np.where(sq > 0, sq, 1.0)):.2e}", flush=True)


@pytest.mark.timeout(900)
def test_batched_full_size_graph_replay():
    prm = batched_tuned() or BATCHED_PARAMS
    nrhs = 8
    print(f"[full-size] batched: generating 64 matrices; plan parameters {prm}", flush=True)
    mats = [A for _, A in matgen.batch_matrices(64)]
    plans = [Plan(A, value_dtype=EHYB_F32, n_rhs=nrhs, lds_bytes=prm["lds_bytes"], halo_rows=prm["halo_rows"],
                  rows_per_wave=prm["rows_per_wave"]).upload("cuda:0") for A in mats]
    B = Batch(plans, nrhs, "cuda:0")
    g = matgen.rng(4999)
    X = [g.uniform(-1.0, 1.0, (A.n_rows, nrhs)) for A in mats]
    Xd = [torch.from_numpy(x[p.perm()].astype(np.float32)).to("cuda:0") for x, p in zip(X, plans)]
    Yd = [torch.empty_like(x) for x in Xd]
    Ye = [torch.empty_like(x) for x in Xd]
    B.spmm(Xd, Ye)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.spmm(Xd, Yd)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        B.spmm(Xd, Yd, stream=s)
    for y in Yd:
        y.fill_(float("nan"))
    graph.replay()
    torch.cuda.synchronize()
    worst = 0.0
    for i, (A, p, x, yd, ye) in enumerate(zip(mats, plans, X, Yd, Ye)):
        assert torch.equal(yd.view(torch.int32), ye.view(torch.int32)), f"matrix {i}: replay differs from eager"
        Aq = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, quantize(A.val, "f32"))
        xq = x.astype(np.float32).astype(np.float64)
        ref = oracle.spmm(Aq, xq)
        sc = oracle.spmm(matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, np.abs(Aq.val)), np.abs(xq))
        got = np.empty_like(ref)
        got[p.perm()] = yd.cpu().numpy()
        err = np.abs(got - ref)
        ok = (err <= gamma32(np.diff(A.row_ptr) + 2.0)[:, None] * sc) | ((sc == 0) & (got == ref))
        assert ok.all(), f"matrix {i} (n={A.n_rows}): {np.count_nonzero(~ok)} entries outside the bound"
        worst = max(worst, float(np.max(err / np.where(sc > 0, sc, 1.0))))
    print(f"[full-size] batched: 64 matrices, worst error / sum|a x| {worst:.2e}", flush=True)
