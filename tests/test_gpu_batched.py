"""GPU parity of the batched multi-matrix, multi-RHS product (one persistent
launch), including repeated launches and HIP graph replays."""
import numpy as np
import pytest

import matgen
import oracle
from oracle.precision import gamma32, quantize
from paper_2204_06666_amd import EHYB_BF16, EHYB_F32, EHYB_F64, Batch, Plan

pytestmark = pytest.mark.gpu

import torch  # noqa: E402


def _mats():
    return [matgen.stencil3d(14, perm_seed=1, val_seed=2),
            matgen.knn_fem(900, perm_seed=3, pt_seed=4, val_seed=5),
            matgen.config_matrix(1),
            matgen.powerlaw(6000, exponent=2.3, mean_deg=8, seed=6),
            matgen.random_small(150, 0.05, 7, empty_rows=10, dense_row=True),
            matgen.stencil3d(9, points=7, val_seed=8)]


def _check(A, X, Y, dt, what):
    m = np.diff(A.row_ptr)
    name = {EHYB_F64: "f64", EHYB_F32: "f32", EHYB_BF16: "bf16"}[dt]
    Aq = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, quantize(A.val, name))
    Xq = X.astype(np.float64) if dt == EHYB_F64 else X.astype(np.float32).astype(np.float64)
    ref = oracle.spmm(Aq, Xq)
    Aabs = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, np.abs(Aq.val))
    s = oracle.spmm(Aabs, np.abs(Xq))
    tol = 1e-12 if dt == EHYB_F64 else gamma32(m + 2)[:, None]
    err = np.abs(Y - ref)
    ok = (err <= tol * s) | ((s == 0) & (Y == ref))
    assert ok.all(), f"{what}: max err {err[~ok].max():.3e}"


def _run(dt, n_rhs, rpw=64, halo=0, lds=160 * 1024):
    mats = _mats()
    # about three partitions per matrix, within the LDS budget of n_rhs-wide rows
    cap = (lds - 64) // (2 * (8 if dt == EHYB_F64 else 4) * n_rhs)
    plans = [Plan(A, value_dtype=dt, n_rhs=n_rhs, rows_per_wave=rpw, halo_rows=halo, lds_bytes=lds,
                  slice_rows=max(64, min(A.n_rows // 3, cap))).upload("cuda:0") for A in mats]
    g = matgen.rng(11)
    X = [g.uniform(-1, 1, (A.n_rows, n_rhs)) for A in mats]
    tdt = torch.float64 if dt == EHYB_F64 else torch.float32
    Xd = [torch.from_numpy(x[p.perm()]).to("cuda:0", tdt).contiguous() for x, p in zip(X, plans)]
    Yd = [torch.empty_like(x) for x in Xd]
    B = Batch(plans, n_rhs)
    B.spmm(Xd, Yd)
    torch.cuda.synchronize()
    return mats, plans, X, Xd, Yd, B


def _unperm(p, Yp):
    Y = np.empty_like(Yp)
    Y[p.perm()] = Yp
    return Y


@pytest.mark.parametrize("dt,n_rhs", [(EHYB_F32, 8), (EHYB_F32, 1), (EHYB_F32, 4), (EHYB_F64, 2),
                                      (EHYB_F64, 8), (EHYB_BF16, 8), (EHYB_BF16, 2)])
@pytest.mark.parametrize("rpw,halo", [(64, 0), (16, -1)])
def test_batched_parity(dt, n_rhs, rpw, halo):
    mats, plans, X, Xd, Yd, B = _run(dt, n_rhs, rpw, halo)
    for A, p, x, y in zip(mats, plans, X, Yd):
        Y = _unperm(p, y.cpu().numpy().astype(np.float64))
        _check(A, x, Y, dt, f"dt={dt} n_rhs={n_rhs} rpw={rpw} halo={halo} n={A.n_rows}")
    print(f"[batched] dt={dt} n_rhs={n_rhs} rpw={rpw} halo={halo} ok", flush=True)


@pytest.mark.parametrize("dt,n_rhs", [(EHYB_F32, 8), (EHYB_F64, 4)])
@pytest.mark.parametrize("lds", [80 * 1024, 53 * 1024, 40 * 1024])
def test_batched_several_workgroups_per_cu(dt, n_rhs, lds):
    """Plans within a half, a third or a quarter of the LDS: the launch runs
    two, three or four workgroups of 8, 5 or 4 wavefronts per CU."""
    mats, plans, X, Xd, Yd, B = _run(dt, n_rhs, lds=lds)
    for A, p, x, y in zip(mats, plans, X, Yd):
        assert p.stats()["lds_bytes_used"] * n_rhs <= lds
        _check(A, x, _unperm(p, y.cpu().numpy().astype(np.float64)), dt, f"{lds} B dt={dt} n_rhs={n_rhs}")


def test_batched_load_modes_identical():
    from paper_2204_06666_amd import EHYB_LOAD_CACHED, EHYB_LOAD_STREAM
    mats, plans, X, Xd, Yd, B = _run(EHYB_F32, 8)
    B.set_load_mode(EHYB_LOAD_CACHED).spmm(Xd, Yd)
    a = [y.clone() for y in Yd]
    B.set_load_mode(EHYB_LOAD_STREAM).spmm(Xd, Yd)
    for u, v in zip(a, Yd):
        assert torch.equal(u.view(torch.int32), v.view(torch.int32))


@pytest.mark.parametrize("dt,n_rhs", [(EHYB_F32, 8), (EHYB_F64, 2), (EHYB_F64, 8), (EHYB_F64, 4), (EHYB_F64, 1),
                                      (EHYB_BF16, 4), (EHYB_F32, 2)])
def test_batched_long_hub_rows(dt, n_rhs):
    """Hub rows with wide residual slices of hundreds of steps, in the
    batched product (n_rhs-wide rows), next to a small matrix: the pieces
    pre-pass with n_rhs sums per piece, results within the bound and the
    same bits on a second launch."""
    mats = [matgen.powerlaw(60000, exponent=2.2, mean_deg=30, seed=5), matgen.stencil3d(12, perm_seed=1, val_seed=2)]
    xb = 8 if dt == EHYB_F64 else 4
    plans = [Plan(A, value_dtype=dt, n_rhs=n_rhs, halo_rows=-1, rows_per_wave=16,
                  slice_rows=min(2000, (160 * 1024 - 64) // (2 * xb * n_rhs))).upload("cuda:0") for A in mats]
    m = np.asarray(plans[0].arrays()["er_meta"]).reshape(-1, 2).astype(np.int64)
    assert (((m[:, 1] >> 31) == 1) & ((m[:, 1] & 0x7FFFFFFF) > 32)).any()
    assert plans[0].stats()["n_er_pieces"] > 0  # summed in pieces before the product
    g = matgen.rng(21)
    X = [g.uniform(-1, 1, (A.n_rows, n_rhs)) for A in mats]
    tdt = torch.float64 if dt == EHYB_F64 else torch.float32
    Xd = [torch.from_numpy(x[p.perm()]).to("cuda:0", tdt).contiguous() for x, p in zip(X, plans)]
    Yd = [torch.empty_like(x) for x in Xd]
    B = Batch(plans, n_rhs)
    B.spmm(Xd, Yd)
    torch.cuda.synchronize()
    for A, p, x, y in zip(mats, plans, X, Yd):
        _check(A, x, _unperm(p, y.cpu().numpy().astype(np.float64)), dt, "batched hub rows")
    first = [y.clone() for y in Yd]
    B.spmm(Xd, Yd)
    for a, b in zip(first, Yd):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.parametrize("dt", [EHYB_F64, EHYB_F32])
def test_batched_hub_rows_match_the_single_product(dt):
    """With one right-hand side, the batched product of plans whose hub rows
    are summed in pieces gives the single product's bits: the same pieces,
    summed in the same order, by the same partition code."""
    mats = [matgen.powerlaw(60000, exponent=2.2, mean_deg=30, seed=5), matgen.stencil3d(12, perm_seed=1, val_seed=2),
            matgen.powerlaw(6000, exponent=2.3, mean_deg=8, seed=6)]
    plans = [Plan(A, value_dtype=dt, halo_rows=-1, rows_per_wave=16, slice_rows=2000).upload("cuda:0") for A in mats]
    assert plans[0].stats()["n_er_pieces"] > 100 and plans[2].stats()["n_er_pieces"] > 0
    g = matgen.rng(31)
    tdt = torch.float64 if dt == EHYB_F64 else torch.float32
    Xd = [torch.from_numpy(g.uniform(-1, 1, (A.n_rows, 1))).to("cuda:0", tdt) for A in mats]
    Yd = [torch.empty_like(x) for x in Xd]
    Batch(plans, 1).spmm(Xd, Yd)
    for A, p, x, y in zip(mats, plans, Xd, Yd):
        ys = p.spmv(x[:, 0])
        torch.cuda.synchronize()
        assert torch.equal(y[:, 0].view(torch.int32 if dt == EHYB_F32 else torch.int64),
                           ys.view(torch.int32 if dt == EHYB_F32 else torch.int64)), f"n={A.n_rows}"
        Xh = np.empty((A.n_rows, 1))
        Xh[p.perm()] = x.cpu().numpy()
        _check(A, Xh, _unperm(p, y.cpu().numpy().astype(np.float64)), dt, "hub rows, one right-hand side")


def test_repeated_launches_identical():
    mats, plans, X, Xd, Yd, B = _run(EHYB_F32, 8)
    first = [y.clone() for y in Yd]
    for _ in range(5):
        B.spmm(Xd, Yd)
        for a, b in zip(first, Yd):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_graph_capture_replays():
    """One launch recorded in a HIP graph; replayed with new inputs between
    replays and eager work in between, each replay checked against an eager
    launch on the same inputs."""
    mats, plans, X, Xd, Yd, B = _run(EHYB_F32, 8)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.spmm(Xd, Yd)        # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        B.spmm(Xd, Yd, stream=s)
    rng = matgen.rng(99)
    Ye = [torch.empty_like(y) for y in Yd]
    for rep in range(4):
        for x in Xd:
            x.copy_(torch.from_numpy(rng.uniform(-1, 1, tuple(x.shape))).to(x))
        g.replay()
        torch.cuda.synchronize()
        B.spmm(Xd, Ye)       # eager reference launch between replays
        torch.cuda.synchronize()
        for a, b in zip(Yd, Ye):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), f"replay {rep}"
    for A, p, x, y in zip(mats, plans, Xd, Yd):
        Xh = np.empty(tuple(x.shape))
        Xh[p.perm()] = x.cpu().numpy()
        _check(A, Xh, _unperm(p, y.cpu().numpy().astype(np.float64)), EHYB_F32, "after replays")
