"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test would fail for a plausible mistake in the oracle: a dropped term
(dense brute force, exact rational), a wrong or transposed index (non-symmetric
random matrices, A e_j = column j), a wrong sign (eigenvector closed form,
integer exactness), a wrong permutation direction (dense P A P^T).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import matgen

U = 2.0 ** -53


def _gamma(m):
    return m * U / (1 - m * U)


@pytest.mark.parametrize("n,density,seed,kw", [
    (1, 1.0, 1, {}),
    (5, 0.6, 2, {}),
    (17, 0.3, 3, {"empty_rows": 3}),
    (33, 0.2, 4, {"dense_row": True}),
    (64, 0.1, 5, {"explicit_zeros": 20, "negative_zero": True}),
    (64, 0.5, 6, {"empty_rows": 10, "dense_row": True}),
])
def test_dense_brute_force(oracle_mod, n, density, seed, kw):
    A = matgen.random_small(n, density, seed, **kw)
    x = matgen.uniform_vector(n, seed + 100)
    y = oracle_mod.spmv(A, x)
    d = matgen.to_dense(A)
    yd = d @ x
    s = np.abs(d) @ np.abs(x)
    m = max(1, int(np.diff(A.row_ptr).max(initial=0)))
    bound = (_gamma(m) + _gamma(n)) * s
    assert np.all(np.abs(y - yd) <= bound), np.max(np.abs(y - yd) - bound)
    # the matrix is not symmetric: a transposed product must be caught
    if n > 4 and not np.allclose(d, d.T):
        assert not np.all(np.abs((d.T @ x) - y) <= bound)


@pytest.mark.parametrize("n,seed", [(12, 11), (80, 12), (200, 13)])
def test_exact_rational(oracle_mod, n, seed):
    A = matgen.random_small(n, 0.15, seed, empty_rows=2, dense_row=True)
    x = matgen.uniform_vector(n, seed + 1)
    y = oracle_mod.spmv(A, x)
    exact = oracle_mod.spmv_exact(A, x)
    s = oracle_mod.abs_scale(A, x)
    for i in range(n):
        m = int(A.row_ptr[i + 1] - A.row_ptr[i])
        err = abs(Fraction(float(y[i])) - exact[i])
        assert err <= Fraction(_gamma(max(m, 1))) * Fraction(float(s[i])) * Fraction(1 + 1e-12)


def test_unit_vectors_give_columns(oracle_mod):
    A = matgen.random_small(40, 0.2, 21, explicit_zeros=5, negative_zero=True)
    d = matgen.to_dense(A)
    for j in range(A.n_cols):
        e = np.zeros(A.n_cols)
        e[j] = 1.0
        y = oracle_mod.spmv(A, e)
        assert np.array_equal(y, d[:, j])   # one nonzero product per row, times 1


def test_ones_give_row_sums(oracle_mod):
    A = matgen.random_small(150, 0.1, 22, empty_rows=4)
    y = oracle_mod.spmv(A, np.ones(A.n_cols))
    ref = np.array([math.fsum(A.val[A.row_ptr[i]:A.row_ptr[i + 1]]) for i in range(A.n_rows)])
    s = oracle_mod.abs_scale(A, np.ones(A.n_cols))
    m = int(np.diff(A.row_ptr).max())
    assert np.all(np.abs(y - ref) <= _gamma(m) * s + 0.5 * np.spacing(np.abs(ref)))


def test_linearity(oracle_mod):
    A = matgen.random_small(120, 0.08, 23)
    x = matgen.uniform_vector(120, 24)
    z = matgen.uniform_vector(120, 25)
    a, b = 0.75, -1.5
    lhs = oracle_mod.spmv(A, a * x + b * z)
    rhs = a * oracle_mod.spmv(A, x) + b * oracle_mod.spmv(A, z)
    s = oracle_mod.abs_scale(A, np.abs(a * x) + np.abs(b * z))
    m = int(np.diff(A.row_ptr).max())
    assert np.all(np.abs(lhs - rhs) <= 4 * _gamma(m + 2) * s)


def test_integer_poisson_exact(oracle_mod):
    A = matgen.poisson2d(32, perm_seed=7)
    x = matgen.integer_vector(A.n_cols, 8)
    y = oracle_mod.spmv(A, x)
    xi = [int(v) for v in x]
    for i in range(A.n_rows):
        acc = 0
        for p in range(A.row_ptr[i], A.row_ptr[i + 1]):
            acc += int(A.val[p]) * xi[A.col[p]]
        assert y[i] == float(acc)


def test_poisson_eigenvector_closed_form(oracle_mod):
    """Dirichlet 5-point Laplacian on 64x64: sin(p pi i/65) sin(q pi j/65) is an
    eigenvector with eigenvalue 4 - 2cos(p pi/65) - 2cos(q pi/65)."""
    nx = 64
    A = matgen.poisson2d(nx)
    i = np.arange(1, nx + 1)
    for p, q in [(1, 1), (3, 7), (64, 2), (33, 33)]:
        # reduce the integer multiple first so the sine arguments stay in [0, 2 pi)
        x = np.outer(np.sin(np.pi * ((p * i) % 130) / 65),
                     np.sin(np.pi * ((q * i) % 130) / 65)).reshape(-1)
        lam = 4 - 2 * np.cos(p * np.pi / 65) - 2 * np.cos(q * np.pi / 65)
        y = oracle_mod.spmv(A, x)
        s = oracle_mod.abs_scale(A, x)
        # rounding of the product plus the (absolute, few-ulp) error of the sines
        assert np.all(np.abs(y - lam * x) <= 64 * U * (s + np.abs(lam * x) + 1.0))
        # a dropped neighbour or a flipped sign would be of the size of |x|
        assert np.max(np.abs(x)) > 0.1


def test_poisson_row_sums_integer():
    """Row sums of the Dirichlet Laplacian: 0 inside, 1 on an edge, 2 at a corner."""
    import oracle
    nx = 64
    A = matgen.poisson2d(nx)
    y = oracle.spmv(A, np.ones(nx * nx)).reshape(nx, nx)
    want = np.zeros((nx, nx))
    want[0, :] += 1
    want[-1, :] += 1
    want[:, 0] += 1
    want[:, -1] += 1
    assert np.array_equal(y, want)


def test_config1_permuted_consistency(oracle_mod):
    """Configuration 1 is the symmetric relabelling of the plain grid: the
    permuted product equals the relabelled plain product (integer data, exact)."""
    plain = matgen.poisson2d(64)
    perm_A = matgen.poisson2d(64, perm_seed=matgen.CONFIG_SEEDS[1])
    lab = matgen.rng(matgen.CONFIG_SEEDS[1]).permutation(64 * 64)
    x = matgen.integer_vector(64 * 64, 31)
    y_plain = oracle_mod.spmv(plain, x)
    xp = np.empty_like(x)
    xp[lab] = x
    y_perm = oracle_mod.spmv(perm_A, xp)
    assert np.array_equal(y_perm[lab], y_plain)


def test_diagonal_and_permutation_matrices(oracle_mod):
    g = matgen.rng(41)
    n = 50
    d = g.uniform(-3, 3, n)
    D = matgen.from_dense(np.diag(d))
    x = matgen.uniform_vector(n, 42)
    assert np.array_equal(oracle_mod.spmv(D, x), d * x)
    p = g.permutation(n)
    Pm = np.zeros((n, n))
    Pm[np.arange(n), p] = 1.0
    assert np.array_equal(oracle_mod.spmv(matgen.from_dense(Pm), x), x[p])


def test_empty_rows_give_positive_zero(oracle_mod):
    A = matgen.random_small(30, 0.2, 51, empty_rows=30)
    y = oracle_mod.spmv(A, matgen.uniform_vector(30, 52))
    assert np.all(y == 0) and not np.signbit(y).any()


def test_spmm_matches_spmv(oracle_mod):
    A = matgen.random_small(70, 0.1, 61)
    X = matgen.rng(62).uniform(-1, 1, (70, 5))
    Y = oracle_mod.spmm(A, X)
    for r in range(5):
        assert np.array_equal(Y[:, r], oracle_mod.spmv(A, np.ascontiguousarray(X[:, r])))


def test_thread_count_does_not_change_bits(oracle_mod):
    A = matgen.stencil3d(12, perm_seed=3, val_seed=4)
    x = matgen.uniform_vector(A.n_cols, 5)
    assert np.array_equal(oracle_mod.spmv(A, x, threads=1), oracle_mod.spmv(A, x, threads=4))


def test_permute_matches_dense(oracle_mod):
    A = matgen.random_small(45, 0.15, 71, empty_rows=2)
    perm = matgen.rng(72).permutation(45)
    B = oracle_mod.permute(A, perm)
    P = np.eye(45)[perm]              # row i of P is e_{perm[i]}
    assert np.array_equal(matgen.to_dense(B), P @ matgen.to_dense(A) @ P.T)
    for i in range(45):
        c = B.col[B.row_ptr[i]:B.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)


def test_permute_composition_and_products(oracle_mod):
    A = matgen.random_small(60, 0.1, 81, integer=True)
    p = matgen.rng(82).permutation(60)
    q = matgen.rng(83).permutation(60)
    B = oracle_mod.permute(oracle_mod.permute(A, p), q)
    C = oracle_mod.permute(A, p[q])
    assert np.array_equal(B.row_ptr, C.row_ptr) and np.array_equal(B.col, C.col)
    assert np.array_equal(B.val, C.val)
    x = matgen.integer_vector(60, 84, bound=1000)
    # (P A P^T)(P x) = P (A x), exact on integers
    assert np.array_equal(oracle_mod.spmv(oracle_mod.permute(A, p), x[p]), oracle_mod.spmv(A, x)[p])


@pytest.mark.parametrize("n,tau,K,vec", [
    (1_000_000, 8, 1, 3907),
    (3_000_000, 8, 1, 11719),
    (4096, 8, 1, 16),
    (5_242_880, 8, 2, 10240),
    (5_242_879, 8, 1, 20480),
    (10_000_000, 4, 1, 39063),
])
def test_eq1_hand_values(oracle_mod, n, tau, K, vec):
    """Eq. 1-2 on 256 compute units with a 160 KiB budget, worked by hand."""
    assert oracle_mod.eq1_rule(n, tau, 256, 160 * 1024) == (K, vec)


def test_eq1_v100_reading(oracle_mod):
    """80 processors (the paper's V100); K*P partitions, multiple of P."""
    K, vec = oracle_mod.eq1_rule(2_000_000, 8, 80, 96 * 1024)
    assert K == 3 and K * 80 * vec >= 2_000_000 and 2_000_000 * 8 / (K * 80) < 96 * 1024
    assert 2_000_000 * 8 / ((K - 1) * 80) >= 96 * 1024


def test_tolerance_helper_flags_errors(oracle_mod):
    y = np.array([1.0, 2.0, 0.0])
    s = np.array([1.0, 1.0, 0.0])
    oracle_mod.assert_close(y, y.copy(), s)
    with pytest.raises(AssertionError):
        oracle_mod.assert_close(y + np.array([0, 1e-11, 0]), y, s)
    with pytest.raises(AssertionError):
        oracle_mod.assert_close(y + np.array([0, 0, 1e-300]), y, s)
    with pytest.raises(AssertionError):
        oracle_mod.assert_close(np.array([np.nan, 2.0, 0.0]), y, s)


def test_scaled_error_hand_values(oracle_mod):
    """|y - ref| / s per row, 0 for an exact match at zero scale, inf for a
    mismatch at zero scale or a NaN on either side."""
    y = np.array([1.5, -2.0, 0.0, 0.0, 7.0, np.nan])
    ref = np.array([1.0, -2.0, 0.0, 1e-300, 7.0, 1.0])
    s = np.array([4.0, 0.5, 0.0, 0.0, 2.0, 1.0])
    e = oracle_mod.scaled_error(y, ref, s)
    assert e[0] == 0.125 and e[1] == 0.0 and e[2] == 0.0 and e[4] == 0.0
    assert np.isinf(e[3]) and np.isinf(e[5])


def test_gamma_matches_fsum_bound(oracle_mod):
    """Worst-case-ish sum: the recursive sum of m values stays within gamma_m of
    the correctly rounded sum."""
    g = matgen.rng(91)
    for m in (3, 27, 400):
        v = g.uniform(-1, 1, m) * 2.0 ** g.integers(-20, 20, m)
        A = matgen.Csr(1, m, np.array([0, m]), np.arange(m, dtype=np.int32), v)
        y = oracle_mod.spmv(A, np.ones(m))[0]
        exact = math.fsum(v)
        assert abs(y - exact) <= _gamma(m) * np.abs(v).sum() + abs(exact) * U
