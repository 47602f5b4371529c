"""Host preprocessing (Alg. 1-2) through the C ABI, checked on the CPU against
the oracle: structure (O3), bit-exact round trip to P A P^T (O2), the layout
interpreter against O1, error paths, plan files, determinism."""
import ctypes
import os

import numpy as np
import pytest

import matgen
import oracle
from oracle.structure import check_plan, layout_spmv
from paper_2204_06666_amd import EhybError, Plan, _abi


def _full_check(A, plan, value_dtype=np.float64, width_cap=None, x_seed=7, x_bytes=8, acc_bytes=None):
    if width_cap is None:
        width_cap = plan.stats()["ell_width_cap"]      # the cap in effect (automatic by default)
    v = plan.arrays()
    st = check_plan(A, v, width_cap=width_cap, value_dtype=value_dtype, x_bytes=x_bytes, acc_bytes=acc_bytes)
    perm = v["perm"]
    # decode == P A P^T, values bit for bit
    rp, ci, val = plan.decode()
    B = oracle.permute(A, perm)
    assert np.array_equal(rp, B.row_ptr) and np.array_equal(ci, B.col)
    from oracle.precision import quantize
    want = quantize(B.val, {np.float64: "f64", np.float32: "f32"}.get(value_dtype, value_dtype))
    assert np.array_equal(val.view(np.uint64), want.view(np.uint64))
    if value_dtype is np.float64:
        x = matgen.uniform_vector(A.n_rows, x_seed)
        yp = layout_spmv(v, x[perm])
        oracle.assert_close(yp, oracle.spmv(A, x)[perm], oracle.abs_scale(A, x)[perm], what="layout")
    return st


CASES = [
    ("cfg1", lambda: matgen.config_matrix(1), {}),
    ("cfg1-rowonly", lambda: matgen.poisson2d(64, perm_seed=1000, row_only=True), {}),
    ("stencil27", lambda: matgen.stencil3d(18, perm_seed=3, val_seed=4), {"slice_rows": 700}),
    ("stencil7-natural", lambda: matgen.stencil3d(16, points=7, perm_seed=5, val_seed=6),
     {"slice_rows": 300, "partitioner": 1}),
    ("knn", lambda: matgen.knn_fem(1500, perm_seed=1, pt_seed=2, val_seed=3), {"slice_rows": 1024}),
    ("powerlaw", lambda: matgen.powerlaw(3000, exponent=2.3, mean_deg=12, seed=9), {"slice_rows": 400}),
    ("edge-small", lambda: matgen.random_small(200, 0.05, 8, empty_rows=20, dense_row=True,
                                               explicit_zeros=15, negative_zero=True),
     {"slice_rows": 33}),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("rpw,halo", [(64, 0), (16, -1), (1, 0), (64, 7)])
def test_plan_structure_and_roundtrip(name, make, kw, rpw, halo):
    A = make()
    P = Plan(A, rows_per_wave=rpw, halo_rows=halo, **kw)
    st = _full_check(A, P)
    s = P.stats()
    assert s["nnz_ell"] == st["nnz_ell"] and s["nnz_er"] == st["nnz_er"]
    assert s["rows_per_slice"] == rpw and s["lanes_per_row"] == 64 // rpw


@pytest.mark.parametrize("cap", [1, 5, 9])
def test_width_cap(cap):
    A = matgen.stencil3d(12, perm_seed=1, val_seed=2)
    P = Plan(A, slice_rows=600, ell_width_cap=cap)
    _full_check(A, P, width_cap=cap)
    assert P.arrays()["row_ell_len"].max() <= cap


def test_integer_layout_exact():
    A = matgen.poisson2d(40, perm_seed=11)
    x = matgen.integer_vector(A.n_rows, 12)
    P = Plan(A, slice_rows=300, rows_per_wave=8)
    v = P.arrays()
    perm = v["perm"]
    assert np.array_equal(layout_spmv(v, x[perm]), oracle.spmv(A, x)[perm])


def test_block_diagonal_has_no_residual():
    """Connected blocks no larger than a partition: a good partitioner cuts no
    edge, so the residual part is empty."""
    A = matgen.block_diagonal([100] * 6, seed=5, density=0.1)
    P = Plan(A, slice_rows=100, imbalance_pct=1, halo_rows=-1)
    st = _full_check(A, P)
    assert st["nnz_er"] == 0


def test_partitioner_beats_scrambled_blocks():
    """Configuration 1 is randomly relabelled: consecutive blocks of the given
    order cut almost everything, the graph partitioner very little."""
    A = matgen.config_matrix(1)
    nat = Plan(A, slice_rows=512, partitioner=1, halo_rows=-1).stats()
    ml = Plan(A, slice_rows=512, halo_rows=-1).stats()
    assert nat["nnz_er"] / nat["nnz"] > 0.5
    assert ml["nnz_er"] / ml["nnz"] < 0.08


def _grid_partition(shape, block, perm_seed):
    """Partition of a relabelled grid (matgen's labelling) into axis-aligned
    boxes of `block` nodes per side: part[label[node]] = box of node."""
    n = int(np.prod(shape))
    lab = matgen._relabel(n, perm_seed)
    coords = np.unravel_index(np.arange(n), shape)
    nb = [s // b for s, b in zip(shape, block)]
    box = np.ravel_multi_index(tuple(c // b for c, b in zip(coords, block)), nb)
    part = np.empty(n, dtype=np.int32)
    part[lab] = box
    return part


def test_partitioner_cut_close_to_geometric_boxes():
    """Closed forms of the cut of box partitions of a grid, and the
    multilevel partitioner measured against them.  With the halo off, the
    residual part holds exactly the entries whose column lies in another
    partition (Section 3.1).  A 5-point 64x64 grid in 2x4 boxes of 32x16 cuts
    64 + 3*64 edges, each stored twice: 512 entries.  In a 27-point m^3 grid,
    a line of length m has 3m - 2 ordered neighbour pairs (offsets -1, 0, +1),
    so the grid holds (3m - 2)^3 entries and a box of side b keeps (3b - 2)^3:
    32^3 in 8^3 boxes cuts 94^3 - 64 * 22^3 = 149112.  The partitioner, blind to
    the geometry, must stay within 1.3x (2-D) and 1.1x (3-D) of these cuts."""
    A = matgen.config_matrix(1)
    geo = Plan(A, slice_rows=512, halo_rows=-1, partition=_grid_partition((64, 64), (32, 16), 1000))
    assert geo.stats()["nparts"] == 8 and geo.stats()["nnz_er"] == 512
    _full_check(A, geo)
    ml = Plan(A, slice_rows=512, halo_rows=-1).stats()
    assert ml["nnz_er"] <= 1.3 * 512, ml["nnz_er"]

    A = matgen.stencil3d(32, perm_seed=7, val_seed=8)
    assert A.nnz == 94 ** 3
    geo = Plan(A, slice_rows=512, halo_rows=-1, partition=_grid_partition((32, 32, 32), (8, 8, 8), 7))
    assert geo.stats()["nparts"] == 64 and geo.stats()["nnz_er"] == 94 ** 3 - 64 * 22 ** 3
    ml = Plan(A, slice_rows=512, halo_rows=-1).stats()
    assert ml["nnz_er"] <= 1.1 * (94 ** 3 - 64 * 22 ** 3), ml["nnz_er"]


def test_eq1_default_slice_rows():
    A = matgen.stencil3d(100, points=7)   # n = 1e6
    n = A.n_rows
    # tau = 16: each partition row keeps its x element and a residual accumulator
    K, vec = oracle.eq1_rule(n, 16, 256, 160 * 1024)
    P = Plan(A, partitioner=1)
    s = P.stats()
    assert s["eq1_K"] == K and s["slice_rows"] == vec == 3907
    assert s["nparts"] == -(-n // vec)
    # small n: the floor at min(n, 512)
    B = matgen.config_matrix(1)
    assert Plan(B, partitioner=1).stats()["slice_rows"] == 512


def test_partition_sizes_within_cap():
    A = matgen.stencil3d(20, perm_seed=2, val_seed=3)
    P = Plan(A, slice_rows=500, imbalance_pct=2)
    ps = P.arrays()["part_start"]
    assert np.diff(ps).max() <= 510
    assert np.diff(ps).min() > 0


def test_determinism_same_seed():
    A = matgen.stencil3d(14, perm_seed=2, val_seed=3)
    a = Plan(A, slice_rows=400, seed=5).arrays()
    b = Plan(A, slice_rows=400, seed=5).arrays()
    for k in ("perm", "part_start", "ell_val", "ell_col", "er_col", "ell_meta", "er_meta", "er_row", "ell_free"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("make", [lambda: matgen.knn_fem(6000, perm_seed=1, pt_seed=2, val_seed=3),
                                  lambda: matgen.powerlaw(30000, exponent=2.3, mean_deg=10, seed=4),
                                  lambda: matgen.stencil3d(24, perm_seed=5, val_seed=6)])
def test_plan_independent_of_thread_count(make):
    """The parallel partitioner and encoder give the same plan for a seed on
    any number of host threads (matching, refinement and bisection tasks are
    scheduled without affecting the result)."""
    A = make()
    ref = Plan(A, n_threads=1, seed=3).arrays()
    for t in (2, 3, 8):
        got = Plan(A, n_threads=t, seed=3).arrays()
        for k in ("perm", "part_start", "halo_idx", "ell_val", "ell_col", "er_col", "ell_meta"):
            assert np.array_equal(ref[k], got[k]), (t, k)


def test_tiny_and_empty():
    for n in (0, 1, 2, 65):
        A = matgen.random_small(n, 0.5, 3) if n else matgen.Csr(0, 0, np.zeros(1, np.int64),
                                                                np.zeros(0, np.int32), np.zeros(0))
        P = Plan(A)
        if n:
            _full_check(A, P)
        assert P.stats()["n"] == n
    A = matgen.random_small(50, 0.0, 1)     # no entries at all
    P = Plan(A, slice_rows=16)
    _full_check(A, P)
    assert P.stats()["nnz"] == 0


@pytest.mark.parametrize("dt,vt,kc", [(1, np.float32, 4), (2, "bf16", 8), (3, np.float32, 4), (4, "bf16", 8)])
@pytest.mark.parametrize("halo", [0, -1])
def test_low_precision_plan_values_rounded(dt, vt, kc, halo):
    """FP32 and BF16 plans (and their binary64-accumulation variants, whose
    residual accumulators take 8 bytes of LDS) store each value rounded to
    nearest even directly from FP64 (checked bit for bit by the oracle's own
    rounding), with 16 bytes of values per lane per step."""
    A = matgen.stencil3d(10, perm_seed=1, val_seed=2)
    P = Plan(A, slice_rows=300, value_dtype=dt, halo_rows=halo)
    assert P.stats()["kc"] == kc
    _full_check(A, P, value_dtype=vt, x_bytes=4, acc_bytes=8 if dt >= 3 else 4)
    v = P.arrays()
    from oracle.precision import quantize
    from oracle.structure import layout_spmv
    x = matgen.uniform_vector(A.n_rows, 3)
    perm = v["perm"]
    Aq = matgen.Csr(A.n_rows, A.n_cols, A.row_ptr, A.col, quantize(A.val, "f32" if dt in (1, 3) else "bf16"))
    yq = oracle.spmv(Aq, x)[perm]
    oracle.assert_close(layout_spmv(v, x[perm]), yq, oracle.abs_scale(Aq, x)[perm], what="quantized layout")


@pytest.mark.parametrize("mutate,status", [
    (lambda A: setattr(A, "n_cols", A.n_cols + 1), _abi.EHYB_EUNSUPPORTED),
    (lambda A: A.col.__setitem__(slice(1, 3), A.col[1:3][::-1].copy()), _abi.EHYB_EINVAL),
    (lambda A: A.col.__setitem__(1, A.col[0]), _abi.EHYB_EINVAL),
    (lambda A: A.col.__setitem__(0, A.n_cols + 5), _abi.EHYB_EINVAL),
    (lambda A: A.col.__setitem__(0, -1), _abi.EHYB_EINVAL),
])
def test_invalid_input_rejected(mutate, status):
    A = matgen.poisson2d(6)
    mutate(A)
    with pytest.raises(EhybError) as e:
        Plan(A)
    assert e.value.status == status


def test_row_ptr_inconsistent():
    A = matgen.poisson2d(6)
    A.row_ptr = A.row_ptr.copy()
    A.row_ptr[3], A.row_ptr[4] = A.row_ptr[4], A.row_ptr[3]
    with pytest.raises(EhybError) as e:
        Plan(A)
    assert e.value.status == _abi.EHYB_EINVAL


@pytest.mark.parametrize("kw", [{"slice_rows": 10241}, {"rows_per_wave": 3}, {"rows_per_wave": 128},
                                {"value_dtype": 7}, {"value_dtype": 5}, {"lds_bytes": 200000}, {"imbalance_pct": -1},
                                {"partitioner": 5}, {"ell_width_cap": -2}])
def test_invalid_params_rejected(kw):
    A = matgen.poisson2d(8)
    with pytest.raises(EhybError) as e:
        Plan(A, **kw)
    assert e.value.status == _abi.EHYB_EINVAL


def test_spmv_before_upload_is_state_error():
    A = matgen.poisson2d(8)
    P = Plan(A)
    lib = _abi.load()
    dummy = ctypes.c_void_p(0x1000)
    st = lib.ehyb_spmv(P.handle, dummy, ctypes.c_void_p(0x2000), 1, None)
    assert st == _abi.EHYB_ESTATE
    assert b"upload" in lib.ehyb_last_error()
    assert lib.ehyb_spmv(P.handle, None, dummy, 1, None) == _abi.EHYB_EINVAL
    assert lib.ehyb_spmv(P.handle, dummy, dummy, 7, None) == _abi.EHYB_EINVAL


def test_save_load_roundtrip(tmp_path):
    A = matgen.stencil3d(12, perm_seed=7, val_seed=8)
    P = Plan(A, slice_rows=500, rows_per_wave=32)
    path = str(tmp_path / "plan.ehyb")
    P.save(path)
    Q = Plan.load(path)
    a, b = P.arrays(), Q.arrays()
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), k
        else:
            assert a[k] == b[k], k
    _full_check(A, Q)
    # corrupt one byte in the middle, and truncate
    raw = bytearray(open(path, "rb").read())
    raw[len(raw) // 2] ^= 0xFF
    bad = str(tmp_path / "bad.ehyb")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(EhybError) as e:
        Plan.load(bad)
    assert e.value.status == _abi.EHYB_EINVAL
    open(bad, "wb").write(open(path, "rb").read()[:100])
    with pytest.raises(EhybError):
        Plan.load(bad)
    with pytest.raises(EhybError):
        Plan.load(str(tmp_path / "missing.ehyb"))


def test_algorithmic_bytes_formula():
    A = matgen.stencil3d(12, perm_seed=1, val_seed=2)
    P = Plan(A, slice_rows=400)
    s = P.stats()
    want = (s["ell_slots"] * 10 + s["er_slots"] * 12 + s["nslices"] * 16
            + s["ner_slices"] * (8 + 2 * s["rows_per_slice"]) + (s["nparts"] + 1) * 16 + s["nparts"] * 4
            + s["n_halo"] * 4 + 2 * s["n"] * 8)
    assert s["algorithmic_bytes"] == want


def test_host_threads_do_not_change_the_plan():
    A = matgen.stencil3d(14, perm_seed=4, val_seed=5)
    a = Plan(A, slice_rows=500, n_threads=1).arrays()
    b = Plan(A, slice_rows=500, n_threads=4).arrays()
    for k in ("perm", "ell_val", "ell_col", "er_val", "er_col", "ell_meta", "er_meta", "er_row"):
        assert np.array_equal(a[k], b[k]), k
    assert os.environ.get("OMP_NUM_THREADS", "") == os.environ.get("OMP_NUM_THREADS", "")


def test_halo_caches_all_neighbours_of_a_stencil():
    """With room in LDS every out-of-partition entry of a stencil is served
    from the halo: the residual part is empty and the halo holds exactly the
    distinct external columns."""
    A = matgen.stencil3d(16, perm_seed=3, val_seed=4)
    P = Plan(A, slice_rows=800)
    st = _full_check(A, P)
    s = P.stats()
    assert s["nnz_er"] == 0 and st["nnz_er"] == 0
    none = Plan(A, slice_rows=800, halo_rows=-1).stats()
    assert s["nnz_halo"] == none["nnz_er"] > 0
    assert none["n_halo"] == 0 and none["nnz_halo"] == 0


def test_halo_cap_keeps_most_referenced_columns():
    A = matgen.stencil3d(14, perm_seed=5, val_seed=6)
    cap = 40
    P = Plan(A, slice_rows=700, halo_rows=cap)
    _full_check(A, P)
    v = P.arrays()
    assert np.diff(v["halo_start"]).max() <= cap
    B = oracle.permute(A, v["perm"])
    ps = v["part_start"]
    rows = np.repeat(np.arange(A.n_rows), np.diff(B.row_ptr))
    for p in range(len(ps) - 1):
        sel = (rows >= ps[p]) & (rows < ps[p + 1])
        c = B.col[sel]
        ext = c[(c < ps[p]) | (c >= ps[p + 1])]
        cols, counts = np.unique(ext, return_counts=True)
        h = v["halo_idx"][v["halo_start"][p]:v["halo_start"][p + 1]]
        inh = np.isin(cols, h)
        assert inh.sum() == min(cap, cols.size)
        if (~inh).any() and inh.any():
            assert counts[inh].min() >= counts[~inh].max()


@pytest.mark.parametrize("sr", [3907, 7800, 10200])
def test_lds_budget_respected_at_the_limit(sr):
    """Plans near the LDS limit must leave room for the kernel's own counters."""
    A = matgen.stencil3d(30, perm_seed=1, val_seed=2)
    P = Plan(A, slice_rows=min(sr, A.n_rows))
    s = P.stats()
    assert s["lds_bytes_used"] <= 160 * 1024 - 64


def test_automatic_width_cap_sends_hub_rows_to_wide_slices():
    """Default plans cap ELL rows at 128 load steps per lane group: only hub
    rows reach it, and their excess runs on wide residual slices; -1 keeps
    the paper's uncapped split."""
    A = matgen.powerlaw(20000, exponent=2.1, mean_deg=20, seed=17)
    lens = np.diff(A.row_ptr)
    for rpw in (64, 8):
        P = Plan(A, slice_rows=2000, rows_per_wave=rpw)
        st = P.stats()
        cap = 128 * (64 // rpw) * 2
        assert st["ell_width_cap"] == cap
        assert lens.max() > cap and st["n_er_wide"] > 0
        arr = P.arrays()
        assert arr["row_ell_len"].max() == cap
        _full_check(A, P)
    Q = Plan(A, slice_rows=2000, ell_width_cap=-1)
    assert Q.stats()["ell_width_cap"] == 0
    _full_check(A, Q, width_cap=0)
    # regular matrices never reach the automatic cap: same plan as uncapped
    B = matgen.stencil3d(14, perm_seed=1, val_seed=2)
    a1, a2 = Plan(B, slice_rows=800).arrays(), Plan(B, slice_rows=800, ell_width_cap=-1).arrays()
    for k in ("perm", "ell_val", "ell_col", "er_col"):
        assert np.array_equal(a1[k], a2[k]), k



def test_acc64_plans_size_lds_for_8_byte_accumulators():
    """Binary64 accumulation: LDS per row = 4-byte x element + 8-byte
    accumulator (aligned), so the largest partition is smaller than for FP32."""
    A = matgen.stencil3d(30, perm_seed=1, val_seed=2)
    lim32 = (160 * 1024 - 64) // 8
    lim64 = (160 * 1024 - 64 - 4) // 12
    Plan(A, value_dtype=3, slice_rows=lim64, halo_rows=-1)
    with pytest.raises(EhybError):
        Plan(A, value_dtype=3, slice_rows=lim64 + 1)
    Plan(A, value_dtype=1, slice_rows=lim32)
    P = Plan(A, value_dtype=4, slice_rows=lim64, halo_rows=-1, imbalance_pct=0)
    st = P.stats()
    assert st["lds_bytes_used"] <= 160 * 1024 - 64
    _full_check(A, P, value_dtype="bf16", x_bytes=4, acc_bytes=8)


def test_wide_slice_pieces(tmp_path):
    """ehyb_spmv sums each wide residual slice in pieces of at most 8 steps:
    their number follows from the slices' step counts, survives a plan file,
    and is zero for a plan without wide slices."""
    A = matgen.powerlaw(20000, exponent=2.2, mean_deg=20, seed=8)
    P = Plan(A, slice_rows=1000, halo_rows=-1, rows_per_wave=16)
    st = P.stats()
    m = np.asarray(P.arrays()["er_meta"]).reshape(-1, 2).astype(np.int64)
    wide = (m[:, 1] >> 31) == 1
    steps = m[:, 1] & 0x7FFFFFFF
    assert st["n_er_wide"] == int(wide.sum()) > 0
    assert st["n_er_pieces"] == int((-(-steps[wide] // 8)).sum())
    assert st["n_er_pieces"] > st["n_er_wide"]
    f = str(tmp_path / "p.bin")
    P.save(f)
    assert Plan.load(f).stats()["n_er_pieces"] == st["n_er_pieces"]
    assert Plan(matgen.stencil3d(12, perm_seed=1, val_seed=2)).stats()["n_er_pieces"] == 0


@pytest.mark.parametrize("seed,n,slice_rows", [(3, 20000, 1000), (7, 60000, 2000), (11, 40000, 0)])
def test_partitions_balance_work_on_power_law(seed, n, slice_rows):
    """Rows at least twice the mean length weigh their ELL-eligible entries
    in the partition balance: on power-law graphs, whose hub rows the
    partitioner keeps together, no partition streams much more ELL work than
    the median one (by rows alone the heaviest held about 4x the median)."""
    A = matgen.powerlaw(n, exponent=2.1, mean_deg=20, seed=seed)
    P = Plan(A, slice_rows=slice_rows)
    _full_check(A, P)
    ar = P.arrays()
    ss, meta = ar["slice_start"], ar["ell_meta"]
    ell = np.array([int((meta[ss[p]:ss[p + 1], 1].astype(np.int64) & 0xFFFF).sum()) for p in range(len(ss) - 1)])
    assert ell.max() <= 1.6 * np.median(ell), (ell.max(), np.median(ell))


def test_work_weights_fall_back_at_the_lds_limit():
    """Partitions already at the LDS row limit leave no room for the weights:
    the plan is built balancing rows, within the limit."""
    A = matgen.powerlaw(30000, exponent=2.1, mean_deg=20, seed=5)
    lim = (160 * 1024 - 64) // 16
    P = Plan(A, slice_rows=lim, imbalance_pct=0)
    _full_check(A, P)
    assert P.stats()["max_part_rows"] <= lim


def test_ell_slices_are_placed_round_by_round():
    """ELL slot ranges follow the documented placement: queue positions 0-15
    of every partition in partition order, then positions 16-31, and so on,
    back to back."""
    A = matgen.stencil3d(30, perm_seed=4, val_seed=5)
    P = Plan(A, slice_rows=1500)
    ar = P.arrays()
    ss, meta = ar["slice_start"], ar["ell_meta"]
    keys, offs, ends = [], [], []
    for p in range(len(ss) - 1):
        for q, s in enumerate(range(ss[p], ss[p + 1])):
            keys.append((q // 16, p, q))
            offs.append(int(meta[s, 0]))
            ends.append(int(meta[s, 0]) + int(meta[s, 1] & 0xFFFF) * 64)
    order = sorted(range(len(keys)), key=lambda k: keys[k])
    assert offs[order[0]] == 0
    assert all(offs[b] == ends[a] for a, b in zip(order, order[1:]))
    assert max(max(ss[p + 1] - ss[p] for p in range(len(ss) - 1)), 0) > 16   # several rounds
