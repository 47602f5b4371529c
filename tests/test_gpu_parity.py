"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerance: per row |y_i - yhat_i| <= 1e-12 * sum_j |a_ij x_j| (exact where the
sum is 0); integer-valued inputs must match bit for bit."""
import numpy as np
import pytest

import matgen
import oracle
from paper_2204_06666_amd import (EHYB_LOAD_CACHED, EHYB_LOAD_STREAM, EhybError, Plan, _abi, cache_flush, csr_spmv,
                                  probe_copy, probe_read)
from paper_2204_06666_amd.workloads import HEADLINE, HEADLINE_PARAMS, PAPER_SPLIT_PARAMS

pytestmark = pytest.mark.gpu
TOL = 1e-12

import torch as _torch  # noqa: E402  (imported at collection: the first import can be slow)


@pytest.fixture(scope="module")
def torch():
    assert _torch.cuda.is_available(), "GPU tests need a GPU"
    return _torch


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _ehyb(torch, A, x, permuted=True, **kw):
    P = Plan(A, **kw).upload("cuda:0")
    perm = P.perm()
    if permuted:
        yp = P.spmv(_dev(torch, x[perm])).cpu().numpy()
        y = np.empty_like(yp)
        y[perm] = yp
    else:
        y = P.spmv(_dev(torch, x), permuted=False).cpu().numpy()
    torch.cuda.synchronize()
    return y, P


def _check(A, x, y, what):
    print(f"[parity] {what} n={A.n_rows} nnz={A.nnz}", flush=True)
    return oracle.assert_close(y, oracle.spmv(A, x), oracle.abs_scale(A, x), TOL, what)


@pytest.mark.parametrize("rpw", [64, 32, 16, 8, 4, 2, 1])
@pytest.mark.parametrize("permuted,halo", [(True, 0), (False, 0), (True, -1)])
def test_config1_parity(torch, rpw, permuted, halo):
    A = matgen.config_matrix(1)
    x = matgen.uniform_vector(A.n_rows, matgen.CONFIG_SEEDS[1] + 2)
    y, _ = _ehyb(torch, A, x, permuted, rows_per_wave=rpw, halo_rows=halo)
    _check(A, x, y, f"cfg1 rpw={rpw} permuted={permuted}")


def _long_wide_slices(P, threshold=32):
    """Wide residual slices (one row on 64 lanes) longer than `threshold` steps."""
    m = np.asarray(P.arrays()["er_meta"]).reshape(-1, 2).astype(np.int64)
    return int((((m[:, 1] >> 31) == 1) & ((m[:, 1] & 0x7FFFFFFF) > threshold)).sum())


@pytest.mark.parametrize("rpw,halo", [(64, 0), (16, -1), (4, 0), (64, -1)])
def test_long_hub_rows(torch, rpw, halo):
    """Residual rows of 10^4 entries (wide slices of hundreds of steps):
    parity with the oracle, and the same bits on every launch."""
    A = matgen.powerlaw(60000, exponent=2.2, mean_deg=30, seed=5)
    x = matgen.uniform_vector(A.n_rows, 6)
    y, P = _ehyb(torch, A, x, rows_per_wave=rpw, halo_rows=halo, slice_rows=2000)
    n_long = _long_wide_slices(P)
    assert n_long > 0
    _check(A, x, y, f"long hub rows rpw={rpw} halo={halo} long wide slices={n_long}")
    xp = _dev(torch, x[P.perm()])
    first = P.spmv(xp).clone()
    for _ in range(5):
        assert torch.equal(P.spmv(xp).view(torch.int64), first.view(torch.int64))


def test_long_hub_rows_unpermuted_and_graph_replays(torch):
    """Hub rows (wide slices summed in pieces by a launch before the product)
    with vectors in the original order, and both launches recorded in a HIP
    graph: every replay, with new x between replays, equals an eager call."""
    A = matgen.powerlaw(30000, exponent=2.1, mean_deg=20, seed=9)
    x = matgen.uniform_vector(A.n_rows, 10)
    P = Plan(A, slice_rows=1500, halo_rows=-1, rows_per_wave=16).upload("cuda:0")
    assert P.stats()["n_er_pieces"] > 0
    xd = _dev(torch, x)
    y = P.spmv(xd, permuted=False)
    torch.cuda.synchronize()
    _check(A, x, y.cpu().numpy(), "hub rows, original order")
    xp = _dev(torch, x[P.perm()])
    yp = torch.empty_like(xp)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        P.spmv(xp, yp, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        P.spmv(xp, yp, stream=s)
    ye = torch.empty_like(yp)
    rng = matgen.rng(12)
    for rep in range(4):
        xp.copy_(torch.from_numpy(rng.uniform(-1, 1, A.n_rows)).to(xp))
        g.replay()
        torch.cuda.synchronize()
        P.spmv(xp, ye)
        torch.cuda.synchronize()
        assert torch.equal(yp.view(torch.int64), ye.view(torch.int64)), f"replay {rep}"


def test_long_hub_rows_integer_exact(torch):
    """Integer values and x: every partial sum is exact, so the product
    equals the oracle bit for bit."""
    A = matgen.powerlaw(60000, exponent=2.2, mean_deg=30, seed=5)
    A = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, np.rint(A.val * 8.0))
    x = matgen.integer_vector(A.n_rows, 19, bound=1 << 10)
    y, P = _ehyb(torch, A, x, rows_per_wave=16, halo_rows=-1, slice_rows=2000)
    assert _long_wide_slices(P) > 0
    assert np.array_equal(y, oracle.spmv(A, x))


@pytest.mark.parametrize("rpw,halo", [(64, 0), (8, -1), (64, -1)])
def test_integer_poisson_bit_exact(torch, rpw, halo):
    A = matgen.config_matrix(1)
    x = matgen.integer_vector(A.n_rows, 77)
    y, _ = _ehyb(torch, A, x, rows_per_wave=rpw, slice_rows=300, halo_rows=halo)
    print(f"[parity] integer poisson rpw={rpw}", flush=True)
    assert np.array_equal(y, oracle.spmv(A, x))


CASES = [
    ("stencil27-30", lambda: matgen.stencil3d(30, perm_seed=5, val_seed=6), {"slice_rows": 2000}),
    ("stencil27-30-small-parts", lambda: matgen.stencil3d(30, perm_seed=5, val_seed=6), {"slice_rows": 130}),
    ("knn", lambda: matgen.knn_fem(3000, perm_seed=1, pt_seed=2, val_seed=3), {"slice_rows": 1500}),
    ("powerlaw", lambda: matgen.powerlaw(20000, exponent=2.2, mean_deg=10, seed=4), {"slice_rows": 2500}),
    ("edge", lambda: matgen.random_small(300, 0.03, 9, empty_rows=30, dense_row=True,
                                         explicit_zeros=20, negative_zero=True), {"slice_rows": 70}),
    ("natural-order", lambda: matgen.stencil3d(24, points=7, val_seed=3), {"slice_rows": 1000, "partitioner": 1}),
    ("width-cap", lambda: matgen.stencil3d(20, perm_seed=1, val_seed=2), {"slice_rows": 900, "ell_width_cap": 7}),
    ("max-slice", lambda: matgen.stencil3d(30, perm_seed=8, val_seed=9), {"slice_rows": 9900, "imbalance_pct": 3}),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("rpw,halo", [(64, 0), (64, -1), (16, 0), (4, -1), (16, 24)])
def test_matrix_families(torch, name, make, kw, rpw, halo):
    A = make()
    x = matgen.uniform_vector(A.n_rows, 123)
    y, P = _ehyb(torch, A, x, rows_per_wave=rpw, halo_rows=halo, **kw)
    st = P.stats()
    _check(A, x, y, f"{name} rpw={rpw} halo={halo} parts={st['nparts']} er={st['nnz_er']}")


@pytest.mark.parametrize("rpw,halo,cap", [(64, -1, 0), (8, -1, 0), (16, 0, 40), (64, 0, 30)])
def test_hub_rows_in_wide_residual_slices(torch, rpw, halo, cap):
    """Power-law matrix with hub rows of thousands of entries: residual rows
    longer than 32 * L entries run on all 64 lanes (wide slices)."""
    A = matgen.powerlaw(40000, exponent=2.1, mean_deg=20, seed=17)
    x = matgen.uniform_vector(A.n_rows, 18)
    y, P = _ehyb(torch, A, x, rows_per_wave=rpw, halo_rows=halo, ell_width_cap=cap, slice_rows=2000)
    st = P.stats()
    assert st["n_er_wide"] > 0
    _check(A, x, y, f"hub rows rpw={rpw} halo={halo} cap={cap} wide={st['n_er_wide']}")


@pytest.mark.parametrize("value_dtype,rows,side", [(0, (160 * 1024 - 64) // 16, 36), (1, (160 * 1024 - 64) // 8, 34)])
def test_largest_partitions(torch, value_dtype, rows, side):
    """Partitions at the LDS limit (x-slice and residual accumulators fill
    the 160 KiB)."""
    A = matgen.stencil3d(side, perm_seed=3, val_seed=4)
    P = Plan(A, slice_rows=rows, imbalance_pct=0, value_dtype=value_dtype).upload("cuda:0")
    st = P.stats()
    assert st["max_part_rows"] <= rows and st["lds_bytes_used"] <= 160 * 1024 - 64
    assert st["max_part_rows"] > 0.9 * rows
    x = matgen.uniform_vector(A.n_rows, 8)
    xd = _dev(torch, x[P.perm()].astype(np.float64 if value_dtype == 0 else np.float32))
    yp = P.spmv(xd).cpu().numpy().astype(np.float64)
    y = np.empty_like(yp)
    y[P.perm()] = yp
    if value_dtype == 0:
        _check(A, x, y, f"largest partitions ({st['max_part_rows']} rows)")
    else:
        from oracle.precision import gamma32, quantize
        Aq = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, quantize(A.val, "f32"))
        xq = x.astype(np.float32).astype(np.float64)
        ref, sc = oracle.spmv(Aq, xq), oracle.abs_scale(Aq, xq)
        assert np.all(np.abs(y - ref) <= gamma32(np.diff(A.row_ptr) + 2) * sc)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 129])
def test_tiny_ragged(torch, n):
    A = matgen.random_small(n, 0.4, n + 3, empty_rows=min(2, n - 1))
    x = matgen.uniform_vector(n, 5)
    y, _ = _ehyb(torch, A, x, slice_rows=max(1, n // 2))
    _check(A, x, y, f"tiny n={n}")


def test_all_empty_rows_give_positive_zero(torch):
    A = matgen.random_small(100, 0.0, 1)
    x = matgen.uniform_vector(100, 2)
    y, _ = _ehyb(torch, A, x, slice_rows=40)
    assert np.all(y == 0) and not np.signbit(y).any()


@pytest.mark.parametrize("halo", [0, -1])
def test_bitwise_determinism(torch, halo):
    A = matgen.stencil3d(40, perm_seed=11, val_seed=12)
    P = Plan(A, slice_rows=3000, halo_rows=halo).upload("cuda:0")
    x = _dev(torch, matgen.uniform_vector(A.n_rows, 13))
    y0 = P.spmv(x).clone()
    for _ in range(20):
        y = P.spmv(x)
        assert torch.equal(y.view(torch.int64), y0.view(torch.int64))
    print("[parity] determinism ok", flush=True)


@pytest.mark.parametrize("value_dtype", [0, 1, 2])
@pytest.mark.parametrize("rpw,halo", [(64, 0), (16, -1)])
def test_load_modes_give_same_bits(torch, value_dtype, rpw, halo):
    """Streaming and plain loads of the value and column arrays: identical
    results, and within the tolerance of the oracle (FP64 plans)."""
    A = matgen.knn_fem(2000, perm_seed=1, pt_seed=2, val_seed=3)
    P = Plan(A, slice_rows=1500, value_dtype=value_dtype, rows_per_wave=rpw, halo_rows=halo).upload("cuda:0")
    x = matgen.uniform_vector(A.n_rows, 5)
    xd = _dev(torch, x[P.perm()].astype(np.float64 if value_dtype == 0 else np.float32))
    yc = P.set_load_mode(EHYB_LOAD_CACHED).spmv(xd).clone()
    ys = P.set_load_mode(EHYB_LOAD_STREAM).spmv(xd).clone()
    P.set_load_mode(0)
    assert torch.equal(yc, ys)
    if value_dtype == 0:
        y = np.empty(A.n_rows)
        y[P.perm()] = ys.cpu().numpy()
        _check(A, x, y, f"stream loads rpw={rpw} halo={halo}")
    with pytest.raises(EhybError):
        P.set_load_mode(3)


def test_plan_file_gives_same_bits(torch, tmp_path):
    A = matgen.stencil3d(16, perm_seed=3, val_seed=4)
    P = Plan(A, slice_rows=1000).upload("cuda:0")
    path = str(tmp_path / "p.ehyb")
    P.save(path)
    Q = Plan.load(path).upload("cuda:0")
    x = _dev(torch, matgen.uniform_vector(A.n_rows, 3))
    assert torch.equal(P.spmv(x), Q.spmv(x))


@pytest.mark.parametrize("lanes", [0, 1, 4, 8, 16, 32, 64])
def test_csr_baseline_parity(torch, lanes):
    A = matgen.stencil3d(30, perm_seed=5, val_seed=6)
    x = matgen.uniform_vector(A.n_rows, 4)
    rp = _dev(torch, A.row_ptr.astype(np.int32))
    y = torch.empty(A.n_rows, dtype=torch.float64, device="cuda:0")
    csr_spmv(rp, _dev(torch, A.col), _dev(torch, A.val), _dev(torch, x), y, lanes)
    _check(A, x, y.cpu().numpy(), f"csr lanes={lanes}")


@pytest.mark.parametrize("lanes", [0, 2, 8, 32])
def test_csr_baseline_long_rows(torch, lanes):
    """Rows of up to 7,546 entries: wavefronts holding a row longer than 1024
    entries sum their rows one at a time on all 64 lanes."""
    A = matgen.powerlaw(n=20000, exponent=2.1, mean_deg=20, seed=3)
    assert int(np.diff(A.row_ptr).max()) > 1024
    x = matgen.uniform_vector(A.n_rows, 4)
    rp = _dev(torch, A.row_ptr.astype(np.int32))
    y = torch.empty(A.n_rows, dtype=torch.float64, device="cuda:0")
    csr_spmv(rp, _dev(torch, A.col), _dev(torch, A.val), _dev(torch, x), y, lanes)
    _check(A, x, y.cpu().numpy(), f"csr long rows lanes={lanes}")


def test_headline_full_size(torch):
    """The benchmarked workload at full size, in the benchmark's launch
    configuration: every row against the oracle."""
    A = matgen.config_matrix(HEADLINE["config"])
    assert A.n_rows == HEADLINE["n"] and A.nnz == HEADLINE["nnz"]
    x = matgen.uniform_vector(A.n_rows, HEADLINE["x_seed"])
    y, P = _ehyb(torch, A, x, **HEADLINE_PARAMS)
    w = _check(A, x, y, "headline")
    print(f"[parity] headline worst scaled error {w:.2e} stats {P.stats()['nparts']} parts", flush=True)
    y2, _ = _ehyb(torch, A, x, permuted=False, **HEADLINE_PARAMS)
    _check(A, x, y2, "headline unpermuted")
    y3, P3 = _ehyb(torch, A, x, **PAPER_SPLIT_PARAMS)
    assert P3.stats()["nnz_er"] > 0
    _check(A, x, y3, "headline, paper split (residual part read from device memory)")
    # the comparator on the same input
    rp = _dev(torch, A.row_ptr.astype(np.int32))
    yc = torch.empty(A.n_rows, dtype=torch.float64, device="cuda:0")
    csr_spmv(rp, _dev(torch, A.col), _dev(torch, A.val), _dev(torch, x), yc, 0)
    _check(A, x, yc.cpu().numpy(), "headline csr")


def test_errors_on_device(torch):
    A = matgen.poisson2d(16)
    P = Plan(A).upload("cuda:0")
    x = torch.zeros(A.n_rows, dtype=torch.float64, device="cuda:0")
    with pytest.raises(EhybError) as e:
        P.spmv(x, x)
    assert e.value.status == _abi.EHYB_EINVAL
    with pytest.raises(ValueError):
        P.spmv(x.float())


def test_probes(torch):
    src = torch.arange(1 << 20, dtype=torch.int32, device="cuda:0")
    dst = torch.zeros_like(src)
    probe_copy(src, dst)
    sink = torch.zeros(65536, dtype=torch.int64, device="cuda:0")
    probe_read(src, sink)
    sink2 = torch.zeros(65536, dtype=torch.int64, device="cuda:0")
    cache_flush(src, sink2)  # the same reduction with cache-allocating loads
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert torch.equal(sink, sink2)
    # the per-workgroup partials of the 32-bit words' XOR combine to the XOR of all words
    w = np.bitwise_xor.reduce(src.cpu().numpy().view(np.uint32))
    assert np.bitwise_xor.reduce(sink.cpu().numpy().astype(np.uint64) & 0xFFFFFFFF) == w
