"""Seeded input generators: closed-form sizes, canonical CSR, determinism."""
import numpy as np
import pytest

import matgen


def _canonical(A):
    assert A.row_ptr[0] == 0 and np.all(np.diff(A.row_ptr) >= 0)
    assert A.row_ptr[-1] == A.col.size == A.val.size
    for i in range(A.n_rows):
        c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    assert A.col.min(initial=0) >= 0 and A.col.max(initial=-1) < A.n_cols


def _sym_pattern(A):
    d = matgen.to_dense(A) != 0
    return np.array_equal(d, d.T)


def test_poisson_sizes():
    for nx in (1, 2, 7, 64):
        A = matgen.poisson2d(nx)
        assert A.nnz == 5 * nx * nx - 4 * nx
    A = matgen.config_matrix(1)
    assert A.n_rows == 4096 and A.nnz == 20224
    _canonical(A)


def test_stencil27_size_and_dominance():
    A = matgen.stencil3d(10, perm_seed=5, val_seed=6)
    assert A.nnz == 28 ** 3          # (3n-2)^3 for the 27-point stencil
    _canonical(A)
    assert _sym_pattern(A)
    d = matgen.to_dense(A)
    off = np.abs(d).sum(axis=1) - np.abs(np.diag(d))
    assert np.all(np.diag(d) > off)
    assert np.abs(d - np.diag(np.diag(d))).max() <= 1.0


def test_stencil7_size():
    A = matgen.stencil3d(6, points=7)
    n = 6
    assert A.nnz == n ** 3 + 6 * n * n * (n - 1)


def test_relabel_is_symmetric_permutation():
    A0 = matgen.stencil3d(5, points=7)
    A1 = matgen.stencil3d(5, points=7, perm_seed=9)
    lab = matgen.rng(9).permutation(125)
    d0 = matgen.to_dense(A0) != 0
    d1 = matgen.to_dense(A1) != 0
    P = np.zeros((125, 125))
    P[lab, np.arange(125)] = 1
    assert np.array_equal(d1, (P @ d0 @ P.T) != 0)


def test_row_only_permutation():
    A = matgen.poisson2d(8, perm_seed=3, row_only=True)
    _canonical(A)
    assert not _sym_pattern(A)


def test_determinism():
    a = matgen.stencil3d(6, perm_seed=1, val_seed=2)
    b = matgen.stencil3d(6, perm_seed=1, val_seed=2)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.val, b.val)
    assert np.array_equal(matgen.uniform_vector(10, 3), matgen.uniform_vector(10, 3))


def test_knn_fem_blocks_and_mutual():
    A = matgen.knn_fem(400, 12, 40, 3, perm_seed=1, pt_seed=2, val_seed=3)
    _canonical(A)
    assert A.n_rows == 1200
    assert _sym_pattern(A)
    d = matgen.to_dense(A) != 0
    # dof blocks: the 3 rows of a node share one pattern, made of whole 3x3 blocks
    blocks = d.reshape(400, 3, 400, 3)
    assert np.all(blocks.all(axis=(1, 3)) == blocks.any(axis=(1, 3)))
    deg = blocks.any(axis=(1, 3)).sum(axis=1) - 1
    assert deg.min() >= 1 and deg.max() <= 40


def test_powerlaw_long_rows():
    A = matgen.powerlaw(5000, exponent=2.2, mean_deg=8, seed=4)
    _canonical(A)
    lens = np.diff(A.row_ptr)
    assert lens.max() > 10 * lens.mean()


@pytest.mark.parametrize("kw", [{"empty_rows": 5}, {"dense_row": True},
                                {"explicit_zeros": 4, "negative_zero": True}])
def test_random_small_variants(kw):
    A = matgen.random_small(20, 0.2, 7, **kw)
    _canonical(A)
    if "empty_rows" in kw:
        assert (np.diff(A.row_ptr) == 0).sum() >= 5
    if "negative_zero" in kw:
        assert np.signbit(A.val[A.val == 0]).any()


def test_block_diagonal_hidden_blocks():
    A = matgen.block_diagonal([30, 50, 20], seed=3)
    _canonical(A)
    assert A.n_rows == 100 and _sym_pattern(A)
