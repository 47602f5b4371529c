"""GPU parity of the FP32 and BF16 value plans (binary32 x and accumulation).

Reference 1 (the bar): the FP64 product of the quantized values with the
binary32-rounded x, computed by the oracle.  The GPU result must agree with it
within the binary32 accumulation bound gamma_{m+2}(2^-24) * sum |a_q x_q| per
row (m entries, plus the residual add and the final rounding).

Reference 2 (stated): the FP64 product of the original matrix and x.  The
error against it is reported and bounded by the value rounding (2^-24 for
binary32, 2^-8 for bfloat16, relative) plus the rounding of x and the
accumulation bound, all relative to sum |a x|.
"""
import numpy as np
import pytest

import matgen
import oracle
from oracle.precision import gamma32, quantize
from paper_2204_06666_amd import EHYB_BF16, EHYB_BF16_ACC64, EHYB_F32, EHYB_F32_ACC64, Plan

pytestmark = pytest.mark.gpu

import torch  # noqa: E402

DT = {EHYB_F32: ("f32", 2.0 ** -24), EHYB_BF16: ("bf16", 2.0 ** -8),
      EHYB_F32_ACC64: ("f32", 2.0 ** -24), EHYB_BF16_ACC64: ("bf16", 2.0 ** -8)}
ACC64 = (EHYB_F32_ACC64, EHYB_BF16_ACC64)


def gamma64(m):
    u = 2.0 ** -53
    m = np.asarray(m, dtype=np.float64)
    return m * u / (1.0 - m * u)


def acc_bound(dt, m):
    """Accumulation bound relative to sum |a_q x_q|: binary32 sums, or binary64
    sums rounded to binary32 once."""
    if dt in ACC64:
        return 2.0 ** -24 + gamma64(m + 2) * (1 + 2.0 ** -24)
    return gamma32(m + 2)


def _run(A, x, dt, permuted=True, **kw):
    P = Plan(A, value_dtype=dt, **kw).upload("cuda:0")
    x32 = x.astype(np.float32)
    if permuted:
        perm = P.perm()
        yp = P.spmv(torch.from_numpy(x32[perm]).to("cuda:0")).cpu().numpy()
        y = np.empty_like(yp)
        y[perm] = yp
    else:
        y = P.spmv(torch.from_numpy(x32).to("cuda:0"), permuted=False).cpu().numpy()
    torch.cuda.synchronize()
    return y.astype(np.float64), P


def _check(A, x, y, dt, what):
    name, uv = DT[dt]
    Aq = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, quantize(A.val, name))
    xq = x.astype(np.float32).astype(np.float64)
    m = np.diff(A.row_ptr)
    yq = oracle.spmv(Aq, xq)
    sq = oracle.abs_scale(Aq, xq)
    err_q = np.abs(y - yq)
    bound_q = acc_bound(dt, m) * sq
    bad = ~((err_q <= bound_q) | ((sq == 0) & (y == yq)))
    assert not bad.any(), f"{what}: row {np.argmax(bad)} err {err_q[bad].max():.3e} vs quantized reference"
    y64 = oracle.spmv(A, x)
    s64 = oracle.abs_scale(A, x)
    scaled = oracle.scaled_error(y, y64, s64)
    bound = uv + 2.0 ** -24 + acc_bound(dt, m) * (1 + uv) * (1 + 2.0 ** -24)
    assert np.all(scaled <= bound * (1 + 1e-6) + (s64 == 0) * 0), f"{what}: error vs FP64 above the bound"
    print(f"[precision] {what}: max scaled error vs FP64 {scaled.max():.3e} "
          f"(bound {np.max(bound):.3e}), vs quantized {np.max(err_q / np.where(sq > 0, sq, 1)):.3e}",
          flush=True)


CASES = [
    ("cfg1", lambda: matgen.config_matrix(1), {"slice_rows": 512}),
    ("stencil27", lambda: matgen.stencil3d(24, perm_seed=5, val_seed=6), {"slice_rows": 1500}),
    ("knn-3dof", lambda: matgen.knn_fem(2500, perm_seed=1, pt_seed=2, val_seed=3), {"slice_rows": 2000}),
    ("powerlaw", lambda: matgen.powerlaw(20000, exponent=2.2, mean_deg=10, seed=4), {"slice_rows": 2500}),
    ("edge", lambda: matgen.random_small(300, 0.03, 9, empty_rows=30, dense_row=True,
                                         explicit_zeros=20, negative_zero=True), {"slice_rows": 70}),
]


@pytest.mark.parametrize("dt", [EHYB_F32, EHYB_BF16, EHYB_F32_ACC64, EHYB_BF16_ACC64])
@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("rpw,halo", [(64, 0), (16, -1), (8, 0)])
def test_low_precision_parity(dt, name, make, kw, rpw, halo):
    A = make()
    x = matgen.uniform_vector(A.n_rows, 321)
    if dt in ACC64:       # 8-byte accumulators: 12 bytes of LDS per partition row
        kw = dict(kw, slice_rows=min(kw["slice_rows"], (160 * 1024 - 68) // 12))
    y, _ = _run(A, x, dt, rows_per_wave=rpw, halo_rows=halo, **kw)
    _check(A, x, y, dt, f"{DT[dt][0]} {name} rpw={rpw} halo={halo}")


@pytest.mark.parametrize("dt", [EHYB_F32, EHYB_BF16])
def test_low_precision_unpermuted(dt):
    A = matgen.stencil3d(20, perm_seed=7, val_seed=8)
    x = matgen.uniform_vector(A.n_rows, 9)
    y, _ = _run(A, x, dt, permuted=False, slice_rows=1200)
    _check(A, x, y, dt, f"{DT[dt][0]} unpermuted")


@pytest.mark.parametrize("dt", [EHYB_F32, EHYB_BF16, EHYB_F32_ACC64, EHYB_BF16_ACC64])
def test_integer_values_exact(dt):
    """Small integers are exact in bfloat16 and their sums in binary32."""
    A = matgen.random_small(400, 0.05, 11, integer=True, empty_rows=5)
    x = matgen.integer_vector(400, 12, bound=1 << 10)
    y, _ = _run(A, x, dt, slice_rows=100, halo_rows=-1)
    assert np.array_equal(y, oracle.spmv(A, x))


@pytest.mark.parametrize("dt", [EHYB_F32, EHYB_BF16, EHYB_BF16_ACC64])
def test_low_precision_deterministic(dt):
    A = matgen.knn_fem(3000, perm_seed=4, pt_seed=5, val_seed=6)
    P = Plan(A, value_dtype=dt, slice_rows=2500).upload("cuda:0")
    x = torch.from_numpy(matgen.uniform_vector(A.n_rows, 7).astype(np.float32)).to("cuda:0")
    y0 = P.spmv(x).clone()
    for _ in range(10):
        assert torch.equal(P.spmv(x).view(torch.int32), y0.view(torch.int32))


@pytest.mark.parametrize("rpw", [64, 8])
def test_acc64_keeps_long_rows_accurate(rpw):
    """Rows of ~1800 entries: with binary64 accumulation the result is the
    binary32 rounding of the exact product of the stored values and x (error
    at most 2^-24 of sum |a_q x_q|); binary32 accumulation is measurably worse
    (by less than a plain running sum would be: the residual part of these
    rows is summed in pieces of at most 512 entries, which blocks the
    accumulation)."""
    g = matgen.rng(77)
    n = 2000
    dense = g.uniform(-1, 1, (n, n)) * (g.random((n, n)) < 0.9)
    A = matgen.from_dense(dense)
    x = matgen.uniform_vector(n, 78)
    errs = {}
    for dt in (EHYB_F32, EHYB_F32_ACC64):
        y, _ = _run(A, x, dt, rows_per_wave=rpw, slice_rows=700, halo_rows=-1)
        Aq = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, quantize(A.val, "f32"))
        xq = x.astype(np.float32).astype(np.float64)
        yq = oracle.spmv(Aq, xq)
        sq = oracle.abs_scale(Aq, xq)
        errs[dt] = float(np.max(np.abs(y - yq) / sq))
    print(f"[precision] long rows rpw={rpw}: binary32 accumulation {errs[EHYB_F32]:.2e}, "
          f"binary64 {errs[EHYB_F32_ACC64]:.2e}", flush=True)
    assert errs[EHYB_F32_ACC64] <= 2.0 ** -24 * 1.001
    assert errs[EHYB_F32] > 2 * errs[EHYB_F32_ACC64]
