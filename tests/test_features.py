"""The 32 sparsity features (C++, parallel) against their definitions written
out in numpy, and preprocessing with a caller-supplied partition."""
import numpy as np
import pytest

import matgen
from oracle.structure import check_plan
from paper_2204_06666_amd import EhybError, Plan, features


def _lq(sorted_v, q):
    return float(sorted_v[int(np.floor(q * (sorted_v.size - 1)))])


def features_ref(A):
    n, nnz = A.n_rows, A.nnz
    r = np.diff(A.row_ptr).astype(np.int64)
    rows = np.repeat(np.arange(n), r)
    j = A.col.astype(np.int64)
    d = np.abs(j - rows)
    m = nnz / n
    s = np.sqrt(np.mean((r - m) ** 2))
    sl = np.sort(r)
    bw = np.zeros(n, np.int64)
    np.maximum.at(bw, rows, d)
    key = set(zip(rows.tolist(), j.tolist()))
    off = [(a, b) for a, b in zip(rows.tolist(), j.tolist()) if a != b]
    sym = sum((b, a) in key for a, b in off) / len(off) if off else 1.0
    blocks = len(set(zip(rows.tolist(), (j // 4096).tolist())))
    nb = (n + 4095) // 4096
    spread = [len(set((j[(rows >= rb * 4096) & (rows < (rb + 1) * 4096)] // 4096).tolist())) / nb
              for rb in range(nb)]
    k = np.arange(1, n + 1)
    top = (n + 99) // 100
    w = _lq(sl, 0.99)
    nz1 = max(nnz, 1)
    f = [np.log2(n), np.log2(nnz + 1), m, s, s / m if m > 0 else 0.0, sl[0], sl[-1], np.log2(sl[-1] + 1),
         _lq(sl, .10), _lq(sl, .25), _lq(sl, .50), _lq(sl, .75), _lq(sl, .90), w,
         np.mean((r - m) ** 3) / s ** 3 if s > 0 else 0.0, np.mean(r == 0), np.mean(r > 2 * m),
         d.sum() / nnz / n if nnz else 0.0, d.max(initial=0) / n, _lq(np.sort(bw), 0.90) / n,
         np.sum(d < 4096) / nz1, blocks / n, np.mean(spread), np.max(spread), sym,
         np.sum(rows == j) / n, np.sum((2 * k - n - 1) * sl) / (n * nnz) if nnz else 0.0,
         sl[n - top:].sum() / nz1, m / 64, np.sum(w - np.minimum(r, w)) / nz1,
         np.sum(np.maximum(r - w, 0)) / nz1, np.sum(rows // 512 == j // 512) / nz1]
    return np.array(f, dtype=np.float64)


CASES = [("poisson", lambda: matgen.poisson2d(70, perm_seed=1)),
         ("poisson-natural", lambda: matgen.poisson2d(90)),
         ("stencil", lambda: matgen.stencil3d(17, perm_seed=2)),
         ("powerlaw", lambda: matgen.powerlaw(9000, exponent=2.2, mean_deg=9, seed=3)),
         ("edge", lambda: matgen.random_small(300, 0.04, 5, empty_rows=40, dense_row=True)),
         ("one", lambda: matgen.random_small(1, 1.0, 6)),
         ("rowonly", lambda: matgen.poisson2d(40, perm_seed=3, row_only=True))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_features_match_definitions(name, make):
    A = make()
    got = features(A).astype(np.float64)
    ref = features_ref(A)
    np.testing.assert_allclose(got, ref.astype(np.float32).astype(np.float64), rtol=2e-6, atol=1e-7,
                               err_msg=name)
    assert np.array_equal(features(A, n_threads=1), features(A, n_threads=5))


def test_feature_values_by_hand():
    """2-D 5-point Poisson on a 3x3 grid, natural order: row lengths
    3,4,3,4,5,4,3,4,3 (m = 33/9), every entry mirrored, diagonal stored."""
    f = features(matgen.poisson2d(3)).astype(np.float64)
    assert f[0] == pytest.approx(np.log2(9)) and f[2] == pytest.approx(33 / 9)
    assert (f[5], f[6], f[10]) == (3, 5, 4)
    assert f[24] == 1.0 and f[25] == 1.0 and f[15] == 0.0
    assert f[20] == 1.0 and f[31] == 1.0 and f[22] == 1.0
    assert f[18] == pytest.approx(3 / 9)   # |i - j| = grid width at most


def test_features_reject_bad_input():
    A = matgen.poisson2d(5)
    A.col[[1, 2]] = A.col[[2, 1]]
    with pytest.raises(EhybError):
        features(A)


def test_reencode_with_given_partition():
    """A plan's partition fed back with other encoding parameters gives a
    valid plan with the same partitions (no re-partitioning)."""
    A = matgen.knn_fem(1500, perm_seed=1, pt_seed=2, val_seed=3)
    base = Plan(A, slice_rows=900)
    part = base.partition()
    for kw in ({"rows_per_wave": 16}, {"ell_width_cap": 20}, {"halo_rows": -1}, {"value_dtype": 1}):
        P = Plan(A, partition=part, **kw)
        assert np.array_equal(P.partition(), part), kw
        check_plan(A, P.arrays(), x_bytes=8 if kw.get("value_dtype", 0) == 0 else 4,
                   width_cap=P.stats()["ell_width_cap"],
                   value_dtype=np.float64 if kw.get("value_dtype", 0) == 0 else np.float32)
        assert P.stats()["slice_rows"] == np.bincount(part).max()


def test_given_partition_validation():
    A = matgen.poisson2d(30)
    n = A.n_rows
    with pytest.raises(EhybError):
        Plan(A, partition=np.full(n, -1))
    with pytest.raises(EhybError):            # one partition above the LDS budget of 256 rows
        Plan(A, partition=np.zeros(n), lds_bytes=2 * 8 * 256 + 64)
    gaps = np.arange(n) // 100 * 3            # ids 0, 3, 6, ...: empty ids dropped
    P = Plan(A, partition=gaps)
    assert P.stats()["nparts"] == (n + 99) // 100
    assert np.array_equal(np.unique(P.partition()), np.arange((n + 99) // 100))
