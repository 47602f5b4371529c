"""CPU oracle for the EHYB SpMV (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never does, and this
package imports nothing from the GPU library: the only code the two sides share
is the seeded input generator module ``matgen``.

Contents (each follows the passage cited in its docstring):

* ``spmv``        O1, plain FP64 CSR product (C, ``spmv_ref.c``), y = A x.
* ``abs_scale``   s_i = sum_j |a_ij||x_j|, the scale of the per-row error bound.
* ``spmm``        O1 applied to several right-hand sides at once.
* ``spmv_exact``  exact rational product (``fractions``) for tiny matrices.
* ``permute``     O2, B = P A P^T for a new->old permutation.
* ``eq1_rule``    Eq. 1 / Eq. 2, the number of partitions and vector-cache size.
* ``check_plan``  O3, structural checker of an EHYB encoding (see ``structure``).
* ``scaled_error`` / ``assert_close``  the per-row tolerance test.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

from .structure import check_plan  # noqa: F401  (O3)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spmv_ref.c")
_LIB = os.path.join(_HERE, "liboracle_spmv.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no contraction of multiply-add)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c99", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        for name in ("oracle_spmv_csr_f64", "oracle_abs_scale_f64"):
            f = getattr(lib, name)
            f.argtypes = [i64, p, p, p, p, p, ctypes.c_int]
            f.restype = ctypes.c_int
        lib.oracle_spmm_csr_f64.argtypes = [i64, p, p, p, ctypes.c_int32, p, p, ctypes.c_int]
        lib.oracle_spmm_csr_f64.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr_arrays(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(A.col, dtype=np.int32)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, ci, v


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def spmv(A, x: np.ndarray, threads: int = 0) -> np.ndarray:
    """O1: y = A x in FP64, each row summed left to right in column order
    (Introduction, definition of SpMV)."""
    lib = _load()
    rp, ci, v = _csr_arrays(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.shape != (A.n_cols,):
        raise ValueError("x has the wrong length")
    y = np.empty(A.n_rows, dtype=np.float64)
    rc = lib.oracle_spmv_csr_f64(A.n_rows, _ptr(rp), _ptr(ci), _ptr(v), _ptr(x), _ptr(y), threads)
    if rc != 0:
        raise RuntimeError("oracle spmv failed")
    return y


def abs_scale(A, x: np.ndarray, threads: int = 0) -> np.ndarray:
    """s_i = sum_j |a_ij| |x_j| (scale of the per-row error bound)."""
    lib = _load()
    rp, ci, v = _csr_arrays(A)
    x = np.ascontiguousarray(x, dtype=np.float64)
    s = np.empty(A.n_rows, dtype=np.float64)
    lib.oracle_abs_scale_f64(A.n_rows, _ptr(rp), _ptr(ci), _ptr(v), _ptr(x), _ptr(s), threads)
    return s


def spmm(A, X: np.ndarray, threads: int = 0) -> np.ndarray:
    """Y = A X for row-major X [n_cols][n_rhs]; one O1 sum per column of X."""
    lib = _load()
    rp, ci, v = _csr_arrays(A)
    X = np.ascontiguousarray(X, dtype=np.float64)
    n_rhs = X.shape[1]
    Y = np.empty((A.n_rows, n_rhs), dtype=np.float64)
    rc = lib.oracle_spmm_csr_f64(A.n_rows, _ptr(rp), _ptr(ci), _ptr(v), n_rhs, _ptr(X), _ptr(Y),
                                 threads)
    if rc != 0:
        raise RuntimeError("oracle spmm failed")
    return Y


def spmv_exact(A, x: np.ndarray) -> list:
    """Exact rational y = A x (every binary64 value is a dyadic rational)."""
    xf = [Fraction(float(t)) for t in x]
    out = []
    for i in range(A.n_rows):
        s = Fraction(0)
        for p in range(int(A.row_ptr[i]), int(A.row_ptr[i + 1])):
            s += Fraction(float(A.val[p])) * xf[int(A.col[p])]
        out.append(s)
    return out


def permute(A, perm: np.ndarray):
    """O2: B = P A P^T for ``perm`` mapping new index -> old index, i.e.
    B[i][j] = A[perm[i]][perm[j]], columns re-sorted within each row.

    The reordering of the method relabels rows and columns with the same
    table (Alg. 1 builds it; Alg. 2 applies it to both rows and columns)."""
    perm = np.asarray(perm, dtype=np.int64)
    n = A.n_rows
    if A.n_cols != n or perm.shape != (n,):
        raise ValueError("permute needs a square matrix and a permutation of its size")
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    if not np.array_equal(np.sort(perm), np.arange(n)):
        raise ValueError("perm is not a permutation")
    lens = np.diff(A.row_ptr)[perm]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    # entry q of new row i comes from position row_ptr_A[perm[i]] + (q - row_ptr[i])
    src = np.repeat(A.row_ptr[:-1][perm] - row_ptr[:-1], lens) + np.arange(row_ptr[-1])
    newcol = inv[A.col[src]]
    newrow = np.repeat(np.arange(n), lens)
    order = np.lexsort((newcol, newrow))
    from matgen import Csr
    return Csr(n, n, row_ptr, newcol[order].astype(np.int32), A.val[src][order].copy())


def eq1_rule(n: int, tau: int, P: int, shm: int):
    """Eq. 1 and Eq. 2: the smallest positive integer K with
    n*tau / (K*P) < SHM, and the vector-cache size VecSize = ceil(n / (K*P)).
    Returns (K, VecSize)."""
    if n <= 0:
        return 1, 0
    K = 1
    while not (n * tau < shm * K * P):
        K += 1
    return K, -(-n // (K * P))


def scaled_error(y: np.ndarray, yref: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Per-row |y - yref| / s, with 0 where both agree exactly and inf where the
    scale is zero but the values differ."""
    y = np.asarray(y, dtype=np.float64)
    yref = np.asarray(yref, dtype=np.float64)
    diff = np.abs(y - yref)
    out = np.zeros_like(diff)
    nz = s > 0
    out[nz] = diff[nz] / s[nz]
    bad = (~nz) & (y != yref)
    out[bad] = np.inf
    nan = np.isnan(y) | np.isnan(yref)
    out[nan] = np.inf
    return out


def assert_close(y, yref, s, tol: float = 1e-12, what: str = "") -> float:
    """|y_i - yref_i| <= tol * s_i for every row i (exact where s_i == 0).
    Returns the largest scaled error."""
    e = scaled_error(y, yref, s)
    worst = float(e.max()) if e.size else 0.0
    if not worst <= tol:
        i = int(np.argmax(e))
        raise AssertionError(
            f"{what}: row {i} scaled error {e[i]:.3e} > {tol:.1e} "
            f"(y={y[i]!r}, ref={yref[i]!r}, scale={s[i]!r})")
    return worst
