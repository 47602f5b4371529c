"""Seeded synthetic sparse matrices and dense vectors.

This module only constructs inputs. It holds none of the SpMV method's
arithmetic (no products, no partitioning, no reordering) and it is shared by
the oracle-side tests and the GPU-side tests and benchmark alike.

Every matrix is returned as canonical CSR in a :class:`Csr` record:
``row_ptr`` int64[n+1], ``col`` int32[nnz] (strictly increasing within a row),
``val`` float64[nnz].

Families (stand-ins for the paper's FEM / CFD / structural matrix classes,
whose SuiteSparse instances are not available here):

* ``poisson2d``   2-D 5-point Dirichlet Laplacian (4 on the diagonal, -1 off).
* ``stencil3d``   3-D 7- or 27-point stencil, off-diagonals ~ U[-1,1], strictly
                  diagonally dominant diagonal ``1 + sum_j |a_ij|``.
* ``knn_fem``     unstructured mesh stand-in: random points in the unit cube,
                  mutual k-nearest-neighbour links with per-point k ~ U{kmin..kmax},
                  ``dof x dof`` blocks per link.
* ``powerlaw``    Chung-Lu random graph with a power-law expected degree
                  sequence (circuit-like long rows).
* ``random_small`` tiny irregular matrices for property tests (empty rows,
                  a dense row, explicit zeros, negative zeros).

Node relabelling: ``perm_seed`` relabels the graph's nodes with a uniformly
random permutation while the matrix is being built (the symmetric P·A·Pᵀ
reading of "rows randomly permuted"); ``row_only=True`` scrambles only the
row order (P·A).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Csr", "rng", "poisson2d", "stencil3d", "knn_fem", "powerlaw", "random_small",
    "uniform_vector", "integer_vector", "block_diagonal", "from_dense", "to_dense",
    "config_matrix", "CONFIG_SEEDS", "batch_matrices", "tuning_matrix",
]


@dataclass
class Csr:
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray  # int64[n_rows+1]
    col: np.ndarray      # int32[nnz]
    val: np.ndarray      # float64[nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.row_ptr)


# Base seed per benchmark configuration: +0 pattern / permutation, +1 values, +2 x.
CONFIG_SEEDS = {1: 1000, 2: 2000, 3: 3000, 4: 4000, 5: 50000}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _relabel(n: int, perm_seed: int | None) -> np.ndarray:
    """label[node] -> new node id (identity when no seed)."""
    if perm_seed is None:
        return np.arange(n, dtype=np.int64)
    return rng(perm_seed).permutation(n).astype(np.int64)


def _assemble_padded(nbr: np.ndarray, vals: np.ndarray, row_label: np.ndarray,
                     col_label_of: np.ndarray, n: int) -> Csr:
    """Build CSR from a padded neighbour table.

    nbr[node, s] is a neighbour node id or -1; vals[node, s] its value.  Row
    ``row_label[node]`` receives the entries, columns are ``col_label_of[nbr]``.
    Columns are sorted within each row.
    """
    valid = nbr >= 0
    cols = np.where(valid, col_label_of[np.where(valid, nbr, 0)], np.iinfo(np.int64).max)
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    valid = np.take_along_axis(valid, order, axis=1)
    counts = valid.sum(axis=1)
    # rows in label order
    node_of_row = np.empty(n, dtype=np.int64)
    node_of_row[row_label] = np.arange(n, dtype=np.int64)
    counts_r = counts[node_of_row]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts_r, out=row_ptr[1:])
    cols_r = cols[node_of_row]
    vals_r = vals[node_of_row]
    valid_r = valid[node_of_row]
    col = cols_r[valid_r].astype(np.int32)
    val = np.ascontiguousarray(vals_r[valid_r], dtype=np.float64)
    return Csr(n, n, row_ptr, col, val)


def poisson2d(nx: int, ny: int | None = None, perm_seed: int | None = None,
              row_only: bool = False) -> Csr:
    """5-point Dirichlet Laplacian on an nx x ny grid: 4 on the diagonal, -1 to
    each in-grid neighbour.  nnz = 5·nx·ny - 2·nx - 2·ny."""
    ny = nx if ny is None else ny
    n = nx * ny
    idx = np.arange(n, dtype=np.int64)
    i, j = idx // ny, idx % ny
    offs = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    nbr = np.full((n, 5), -1, dtype=np.int64)
    vals = np.zeros((n, 5), dtype=np.float64)
    for s, (di, dj) in enumerate(offs):
        ii, jj = i + di, j + dj
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
        nbr[ok, s] = (ii * ny + jj)[ok]
        vals[ok, s] = 4.0 if s == 0 else -1.0
    lab = _relabel(n, perm_seed)
    if row_only:
        return _assemble_padded(nbr, vals, lab, np.arange(n, dtype=np.int64), n)
    return _assemble_padded(nbr, vals, lab, lab, n)


def stencil3d(nx: int, ny: int | None = None, nz: int | None = None, points: int = 27,
              perm_seed: int | None = None, val_seed: int = 0) -> Csr:
    """3-D grid stencil (7 or 27 points).  Off-diagonal values ~ U[-1,1] drawn
    per stored entry in final CSR order; diagonal = 1 + sum of |off-diagonal|
    of its row (strict diagonal dominance)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    idx = np.arange(n, dtype=np.int64)
    i, j, k = idx // (ny * nz), (idx // nz) % ny, idx % nz
    if points == 27:
        offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    elif points == 7:
        offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    else:
        raise ValueError("points must be 7 or 27")
    nbr = np.full((n, len(offs)), -1, dtype=np.int64)
    for s, (a, b, c) in enumerate(offs):
        ii, jj, kk = i + a, j + b, k + c
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (kk >= 0) & (kk < nz)
        nbr[ok, s] = ((ii * ny + jj) * nz + kk)[ok]
    lab = _relabel(n, perm_seed)
    A = _assemble_padded(nbr, np.zeros(nbr.shape), lab, lab, n)
    _fill_dominant(A, val_seed)
    return A


def _fill_dominant(A: Csr, val_seed: int) -> None:
    """Off-diagonals ~ U[-1,1] (one draw per stored entry, CSR order); the
    diagonal is then set to 1 + sum |off-diagonal| of the row."""
    g = rng(val_seed)
    v = g.uniform(-1.0, 1.0, A.nnz)
    rows = np.repeat(np.arange(A.n_rows, dtype=np.int64), np.diff(A.row_ptr))
    diag = A.col.astype(np.int64) == rows
    v[diag] = 0.0
    s = np.bincount(rows, weights=np.abs(v), minlength=A.n_rows)
    v[diag] = 1.0 + s[rows[diag]]
    A.val = v


def knn_fem(npts: int, kmin: int = 12, kmax: int = 40, dof: int = 3,
            perm_seed: int | None = None, pt_seed: int = 0, val_seed: int = 1) -> Csr:
    """Unstructured FEM-like matrix.

    ``npts`` points ~ U[0,1]^3; point p asks for k_p ~ U{kmin..kmax} nearest
    neighbours; an undirected link (p,q) exists when each is among the other's
    k nearest (mutual kNN).  Each node carries ``dof`` unknowns, so every link
    (and the node itself) contributes a dense dof x dof block.  Node labels are
    relabelled by ``perm_seed``; the dof of a node stay consecutive.
    Off-diagonal values ~ U[-1,1]; diagonal made strictly dominant.
    """
    from scipy.spatial import cKDTree

    g = rng(pt_seed)
    pts = g.random((npts, 3))
    kk = g.integers(kmin, kmax + 1, size=npts)
    tree = cKDTree(pts)
    _, nb = tree.query(pts, k=kmax + 1, workers=-1)
    nb = nb[:, 1:].astype(np.int64)  # drop self
    rank_ok = np.arange(kmax)[None, :] < kk[:, None]
    # directed candidate links p->q kept when q in kNN_p(k_p)
    p_idx = np.repeat(np.arange(npts, dtype=np.int64), kmax).reshape(npts, kmax)
    src, dst = p_idx[rank_ok], nb[rank_ok]
    key_fwd = src * npts + dst
    key_rev = dst * npts + src
    key_fwd_sorted = np.sort(key_fwd)
    pos = np.searchsorted(key_fwd_sorted, key_rev)
    pos = np.minimum(pos, key_fwd_sorted.size - 1)
    mutual = key_fwd_sorted[pos] == key_rev
    src, dst = src[mutual], dst[mutual]   # symmetric set: both directions present
    lab = _relabel(npts, perm_seed)
    # node-level adjacency incl. self loop
    s_all = np.concatenate([lab[src], np.arange(npts, dtype=np.int64)])
    d_all = np.concatenate([lab[dst], np.arange(npts, dtype=np.int64)])
    order = np.lexsort((d_all, s_all))
    s_all, d_all = s_all[order], d_all[order]
    node_deg = np.bincount(s_all, minlength=npts)
    # expand to dof blocks: row (s*dof + a) has columns (d*dof + b) for b < dof
    n = npts * dof
    row_len = np.repeat(node_deg * dof, dof)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    node_ptr = np.zeros(npts + 1, dtype=np.int64)
    np.cumsum(node_deg, out=node_ptr[1:])
    node_cols = (d_all[:, None] * dof + np.arange(dof)[None, :]).reshape(-1)
    row_node = np.repeat(np.arange(npts, dtype=np.int64), dof)
    # row r = s*dof + a repeats node s's column segment [node_ptr[s]*dof, node_ptr[s+1]*dof)
    shift = node_ptr[:-1][row_node] * dof - row_ptr[:-1]
    col = node_cols[np.repeat(shift, row_len) + np.arange(row_ptr[-1], dtype=np.int64)]
    col = col.astype(np.int32)
    A = Csr(n, n, row_ptr, col, np.zeros(col.size))
    _fill_dominant(A, val_seed)
    return A


def powerlaw(n: int, exponent: float = 2.5, mean_deg: float = 10.0, seed: int = 0,
             max_deg: int | None = None) -> Csr:
    """Chung-Lu graph: expected degree w_i ∝ i^(-1/(exponent-1)), scaled to the
    requested mean; edges sampled by endpoint-weighted draws (duplicates merged),
    symmetric pattern plus a dominant diagonal.  Labels are random."""
    g = rng(seed)
    i = np.arange(1, n + 1, dtype=np.float64)
    w = i ** (-1.0 / (exponent - 1.0))
    w *= mean_deg * n / w.sum()
    if max_deg is not None:
        w = np.minimum(w, max_deg)
    m = int(round(w.sum() / 2))
    p = w / w.sum()
    a = g.choice(n, size=m, p=p)
    b = g.choice(n, size=m, p=p)
    keep = a != b
    a, b = a[keep], b[keep]
    lab = g.permutation(n)
    a, b = lab[a], lab[b]
    s = np.concatenate([a, b, np.arange(n)])
    d = np.concatenate([b, a, np.arange(n)])
    key = np.unique(s.astype(np.int64) * n + d)
    s, d = key // n, key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(s, minlength=n), out=row_ptr[1:])
    A = Csr(n, n, row_ptr, d.astype(np.int32), np.zeros(d.size))
    _fill_dominant(A, seed + 1)
    return A


def random_small(n: int, density: float, seed: int, empty_rows: int = 0,
                 dense_row: bool = False, explicit_zeros: int = 0,
                 negative_zero: bool = False, integer: bool = False) -> Csr:
    """Small irregular square matrix for property tests."""
    g = rng(seed)
    mask = g.random((n, n)) < density
    if dense_row and n > 0:
        mask[g.integers(n)] = True
    if empty_rows:
        mask[g.choice(n, size=min(empty_rows, n), replace=False)] = False
    if integer:
        dense = g.integers(-8, 9, size=(n, n)).astype(np.float64)
        dense[dense == 0] = 1.0
    else:
        dense = g.uniform(-1.0, 1.0, size=(n, n))
    dense[~mask] = 0.0
    A = from_dense(dense, mask)
    if explicit_zeros and A.nnz:
        z = g.choice(A.nnz, size=min(explicit_zeros, A.nnz), replace=False)
        A.val[z] = 0.0
        if negative_zero:
            A.val[z[: max(1, len(z) // 2)]] = -0.0
    return A


def block_diagonal(block_sizes, seed: int, density: float = 0.5, shuffle: bool = True) -> Csr:
    """Block-diagonal matrix with dense-ish connected blocks, node labels
    shuffled so the block structure is hidden."""
    g = rng(seed)
    n = int(sum(block_sizes))
    dense = np.zeros((n, n))
    mask = np.zeros((n, n), dtype=bool)
    o = 0
    for b in block_sizes:
        m = g.random((b, b)) < density
        m |= m.T
        # chain keeps each block connected
        for t in range(b - 1):
            m[t, t + 1] = m[t + 1, t] = True
        np.fill_diagonal(m, True)
        mask[o:o + b, o:o + b] = m
        dense[o:o + b, o:o + b] = g.uniform(-1, 1, (b, b))
        o += b
    dense[~mask] = 0.0
    if shuffle:
        p = g.permutation(n)
        dense = dense[np.ix_(p, p)]
        mask = mask[np.ix_(p, p)]
    return from_dense(dense, mask)


def from_dense(dense: np.ndarray, mask: np.ndarray | None = None) -> Csr:
    if mask is None:
        mask = dense != 0
    n_rows, n_cols = dense.shape
    r, c = np.nonzero(mask)
    row_ptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n_rows), out=row_ptr[1:])
    return Csr(n_rows, n_cols, row_ptr, c.astype(np.int32),
               np.ascontiguousarray(dense[r, c], dtype=np.float64))


def to_dense(A: Csr) -> np.ndarray:
    d = np.zeros((A.n_rows, A.n_cols))
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
    d[rows, A.col] = A.val
    return d


def uniform_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0,
                   dtype=np.float64) -> np.ndarray:
    return rng(seed).uniform(lo, hi, n).astype(dtype)


def integer_vector(n: int, seed: int, bound: int = 1 << 20) -> np.ndarray:
    return rng(seed).integers(-bound, bound + 1, n).astype(np.float64)


def config_matrix(cfg: int, scale: float = 1.0) -> Csr:
    """Matrices of the benchmark configurations.

    1: 64x64 5-point Poisson, symmetric random relabelling (seed 1000).
    2: 100^3 27-point stencil, U[-1,1] off-diagonals, dominant diagonal,
       random relabelling (seeds 2000/2001).
    3: mutual-kNN FEM stand-in, 1e6 points x 3 dof (``scale`` shrinks it).
    """
    s = CONFIG_SEEDS[cfg]
    if cfg == 1:
        return poisson2d(64, perm_seed=s)
    if cfg == 2:
        m = max(2, int(round(100 * scale ** (1 / 3))))
        return stencil3d(m, points=27, perm_seed=s, val_seed=s + 1)
    if cfg == 3:
        return knn_fem(max(100, int(1_000_000 * scale)), 12, 40, 3,
                       perm_seed=s, pt_seed=s + 3, val_seed=s + 1)
    raise ValueError(f"no matrix recipe for configuration {cfg}")


def batch_matrices(count: int = 64, seed: int = 4000, n_lo: int = 10_000, n_hi: int = 500_000):
    """The uneven batch: matrix i draws, from generator seed + i, a row count
    n ~ log-uniform [n_lo, n_hi] and a family uniformly among the 2-D 5-point
    Poisson (side round(sqrt n)), the 27-point 3-D stencil (side round(cbrt n))
    and the mutual-kNN FEM matrix with 3 dof (n/3 points); every matrix is
    randomly relabelled.  Returns [(family, Csr)]."""
    out = []
    for i in range(count):
        s = seed + i
        g = rng(s)
        n = int(round(np.exp(g.uniform(np.log(n_lo), np.log(n_hi)))))
        fam = ("poisson2d", "stencil27", "knn3")[int(g.integers(0, 3))]
        if fam == "poisson2d":
            A = poisson2d(max(2, int(round(np.sqrt(n)))), perm_seed=s)
        elif fam == "stencil27":
            A = stencil3d(max(2, int(round(n ** (1.0 / 3.0)))), perm_seed=s, val_seed=s + 100_000)
        else:
            A = knn_fem(max(50, n // 3), perm_seed=s, pt_seed=s + 200_000, val_seed=s + 100_000)
        out.append((fam, A))
    return out


def tuning_matrix(i: int, n_lo: int = 10_000, n_hi: int = 1_000_000, seed: int = 50_000):
    """Matrix i of the tuning set, from generator seed + i: n ~ log-uniform
    [n_lo, n_hi]; family uniform among
      stencil  - 2-D 5-point, 3-D 7-point or 3-D 27-point, grid sides drawn
                 with aspect ratios ~ U[0.5, 2];
      knn      - mutual-kNN FEM matrix, k ~ U{12..40}, 1 or 3 dof per point;
      powerlaw - Chung-Lu, exponent ~ U[2.1, 3.0], mean degree ~ U[5, 50];
    every matrix randomly relabelled.  Returns (description, Csr)."""
    s = seed + i
    g = rng(s)
    n = float(np.exp(g.uniform(np.log(n_lo), np.log(n_hi))))
    fam = ("stencil", "knn", "powerlaw")[int(g.integers(0, 3))]
    if fam == "stencil":
        kind = ("2d5", "3d7", "3d27")[int(g.integers(0, 3))]
        if kind == "2d5":
            r = g.uniform(0.5, 2.0)
            nx = max(2, int(round(np.sqrt(n * r))))
            ny = max(2, int(round(n / nx)))
            return f"stencil-2d5 {nx}x{ny}", poisson2d(nx, ny, perm_seed=s)
        r1, r2 = g.uniform(0.5, 2.0, 2)
        nx = max(2, int(round((n * r1 * r1 / r2) ** (1 / 3))))
        ny = max(2, int(round(nx * r2 / r1)))
        nz = max(2, int(round(n / (nx * ny))))
        pts = 7 if kind == "3d7" else 27
        return f"stencil-3d{pts} {nx}x{ny}x{nz}", stencil3d(nx, ny, nz, points=pts, perm_seed=s,
                                                            val_seed=s + 100_000)
    if fam == "knn":
        dof = (1, 3)[int(g.integers(0, 2))]
        npts = max(100, int(round(n / dof)))
        return f"knn dof={dof} pts={npts}", knn_fem(npts, dof=dof, perm_seed=s, pt_seed=s + 200_000,
                                                   val_seed=s + 100_000)
    ex = float(g.uniform(2.1, 3.0))
    md = float(g.uniform(5.0, 50.0))
    return f"powerlaw exp={ex:.3f} deg={md:.1f}", powerlaw(int(round(n)), exponent=ex, mean_deg=md,
                                                           seed=s + 300_000)
