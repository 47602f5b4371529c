"""O3: structural checker of an EHYB encoding (test infrastructure only).

An independent reader of the EHYB arrays.  It re-derives, from the layout
rules alone, which stored slot holds which matrix entry, and then checks the
properties the paper fixes for the format:

* the row permutation is a bijection, and rows of one partition are contiguous
  (Section 3.1: partitions own blocks of rows; Alg. 1 builds the reorder table);
* every partition's slice of x fits the on-chip cache and its local column
  indices fit 16 bits (Section 3.3, Eq. 1-2; Section 3.4, compact index);
* every stored entry of the ELL part has its column inside the row's own
  partition, and (with no width cap) every intra-partition entry is in the ELL
  part, every other entry in the residual ("extra rows") part (Section 3.1-3.2,
  Alg. 1 classification);
* within a partition, rows are ordered by non-increasing ELL entry count
  (Section 3.2, post-partitioning reordering), ties broken by original index;
* padding slots hold +0.0 and a valid column;
* the union of both parts is exactly P A P^T, values bit for bit (the reorder
  of Alg. 2 moves values without touching them).

Layout rules being checked (row-slice = C = 64 / L consecutive permuted rows,
one 64-lane wavefront per row-slice, L lanes per row, KC consecutive entries
per lane per step):

    entry k of row r (0 <= r < C) of row-slice s lives at
        t = k // (L*KC), u = (k // KC) % L, c = k % KC, lane = r*L + u,
        slot = off[s] + (t*64 + lane)*KC + c,
    with (off, steps) = (ell_off, ell_steps) and KC = kc for the ELL part, and
    (er_off, er_steps) with KC = 1 for the residual part.

``view`` is a mapping with the keys: n, nparts, L, kc, perm, part_start,
slice_start, slice_meta (uint32 [nslices, 4]: ell_off, ell_steps, er_off,
er_steps), ell_val, ell_col (uint16), er_val, er_col (int32), row_ell_len,
row_er_len.
"""
from __future__ import annotations

import numpy as np


class PlanError(AssertionError):
    pass


def _req(cond, msg):
    if not cond:
        raise PlanError(msg)


def _slots(view, which: str):
    """Enumerate every slot of one part.

    Returns (slot, row, k, valid): the slot index, the permuted row it belongs
    to (-1 for lanes past the partition end), the entry position within the
    row, and whether it holds a real entry."""
    L = int(view["L"])
    C = 64 // L
    kc = int(view["kc"]) if which == "ell" else 1
    meta = np.asarray(view["slice_meta"], dtype=np.int64).reshape(-1, 4)
    off = meta[:, 0] if which == "ell" else meta[:, 2]
    steps = meta[:, 1] if which == "ell" else meta[:, 3]
    rowlen = np.asarray(view["row_ell_len"] if which == "ell" else view["row_er_len"],
                        dtype=np.int64)
    part_start = np.asarray(view["part_start"], dtype=np.int64)
    slice_start = np.asarray(view["slice_start"], dtype=np.int64)
    nslices = meta.shape[0]
    # partition and first row of each slice
    part_of_slice = np.repeat(np.arange(len(part_start) - 1), np.diff(slice_start))
    _req(part_of_slice.size == nslices, "slice_start does not cover slice_meta")
    row0 = part_start[part_of_slice] + (np.arange(nslices) - slice_start[part_of_slice]) * C
    row_end = part_start[part_of_slice + 1]
    per = steps * 64 * kc
    total = int(per.sum())
    s_of = np.repeat(np.arange(nslices), per)
    o = np.arange(total) - np.repeat(np.cumsum(per) - per, per)
    t = o // (64 * kc)
    lane = (o // kc) % 64
    c = o % kc
    r = lane // L
    u = lane % L
    k = (t * L + u) * kc + c
    row = row0[s_of] + r
    exists = row < row_end[s_of]
    row = np.where(exists, row, -1)
    valid = exists.copy()
    valid[exists] = k[exists] < rowlen[row[exists]]
    slot = off[s_of] + o
    return slot, row, k, valid, part_of_slice[s_of]


def layout_entries(view):
    """(row, col, val, in_ell) of every real stored entry, in permuted indices."""
    part_start = np.asarray(view["part_start"], dtype=np.int64)
    out = []
    for which in ("ell", "er"):
        slot, row, k, valid, part = _slots(view, which)
        vals = np.asarray(view["ell_val" if which == "ell" else "er_val"])
        cols = np.asarray(view["ell_col" if which == "ell" else "er_col"])
        sv = slot[valid]
        col = cols[sv].astype(np.int64)
        if which == "ell":
            col = col + part_start[part[valid]]
        out.append((row[valid], col, vals[sv], np.full(sv.size, which == "ell")))
    return tuple(np.concatenate([o[i] for o in out]) for i in range(4))


def layout_spmv(view, xp: np.ndarray) -> np.ndarray:
    """Execute the EHYB arrays as laid out (a sequential format interpreter):
    y_p = sum over real slots of the row of val * xp[col], in permuted space."""
    row, col, val, _ = layout_entries(view)
    n = int(view["n"])
    return np.bincount(row, weights=val.astype(np.float64) * xp[col], minlength=n)


def check_plan(A, view, tau_x: int = 8, lds_budget: int = 160 * 1024, width_cap: int = 0,
               value_dtype=np.float64, Bperm=None) -> dict:
    """Check every structural property of an EHYB encoding of ``A``.

    ``value_dtype`` is the storage type of values (float64 plans must reproduce
    A's bits; lower-precision plans must reproduce A's values rounded to that
    type).  ``Bperm`` may pass a precomputed P A P^T.  Returns statistics."""
    from . import permute

    n = int(view["n"])
    perm = np.asarray(view["perm"], dtype=np.int64)
    _req(perm.shape == (n,), "perm has the wrong length")
    _req(np.array_equal(np.sort(perm), np.arange(n)), "perm is not a bijection")

    part_start = np.asarray(view["part_start"], dtype=np.int64)
    nparts = int(view["nparts"])
    _req(part_start.shape == (nparts + 1,), "part_start length")
    _req(part_start[0] == 0 and part_start[-1] == n, "partitions must cover all rows")
    sizes = np.diff(part_start)
    _req(n == 0 or (sizes > 0).all(), "empty partition")
    _req((sizes <= 65536).all(), "partition larger than a 16-bit local index allows")
    _req((sizes * tau_x <= lds_budget).all(), "x-slice exceeds the on-chip budget")

    L = int(view["L"])
    _req(L in (1, 2, 4, 8, 16, 32, 64), "lanes per row must divide 64")
    C = 64 // L
    slice_start = np.asarray(view["slice_start"], dtype=np.int64)
    _req(np.array_equal(np.diff(slice_start), -(-sizes // C)), "slices per partition")

    meta = np.asarray(view["slice_meta"], dtype=np.int64).reshape(-1, 4)
    kc = int(view["kc"])
    ell_val = np.asarray(view["ell_val"])
    er_val = np.asarray(view["er_val"])
    ell_col = np.asarray(view["ell_col"])
    er_col = np.asarray(view["er_col"])
    _req(ell_col.dtype == np.uint16, "ELL columns must be 16-bit")
    # slot ranges inside the arrays and disjoint
    for off, steps, arr, width in ((meta[:, 0], meta[:, 1], ell_val, 64 * kc),
                                   (meta[:, 2], meta[:, 3], er_val, 64)):
        end = off + steps * width
        _req((end <= arr.size).all(), "slot range past the end of its array")
        o = np.argsort(off, kind="stable")
        nz = steps[o] > 0
        _req((off[o][nz][1:] >= end[o][nz][:-1]).all(), "overlapping slot ranges")

    row_ell_len = np.asarray(view["row_ell_len"], dtype=np.int64)
    row_er_len = np.asarray(view["row_er_len"], dtype=np.int64)
    part_of_row = np.repeat(np.arange(nparts), sizes)

    # minimal widths: each slice's step count is what its longest row needs
    for lens, steps, per in ((row_ell_len, meta[:, 1], L * kc), (row_er_len, meta[:, 3], L)):
        if n:
            need = np.zeros(meta.shape[0], dtype=np.int64)
            slice_of_row = slice_start[part_of_row] + (np.arange(n) - part_start[part_of_row]) // C
            np.maximum.at(need, slice_of_row, lens)
            _req(np.array_equal(steps, -(-need // per)), "slice width is not its longest row")

    # padding slots
    for which, vals, cols in (("ell", ell_val, ell_col), ("er", er_val, er_col)):
        slot, row, k, valid, part = _slots(view, which)
        pad = slot[~valid]
        bits = np.ascontiguousarray(vals[pad]).view(np.uint8)
        _req(not bits.any(), f"{which} padding slot is not +0.0")
        pc = cols[pad].astype(np.int64)
        if which == "ell":
            _req((pc < sizes[part[~valid]]).all(), "ELL padding column outside its slice")
            rv = row[valid]
            _req((cols[slot[valid]].astype(np.int64) < sizes[part_of_row[rv]]).all(),
                 "ELL local column outside its partition")
        else:
            _req(((pc >= 0) & (pc < n)).all(), "residual padding column out of range")

    row, col, val, in_ell = layout_entries(view)
    _req(((col >= 0) & (col < n)).all(), "column out of range")
    same = part_of_row[row] == part_of_row[col]
    _req(same[in_ell].all(), "ELL entry whose column is outside the row's partition")
    if width_cap == 0:
        _req((~same[~in_ell]).all(), "intra-partition entry left in the residual part")
    else:
        _req((row_ell_len <= width_cap).all(), "ELL row longer than the width cap")
        spill = ~in_ell & same
        _req((row_ell_len[row[spill]] == width_cap).all(),
             "intra-partition entry spilled from a row below the cap")

    # ordering inside partitions: non-increasing ELL count, ties by original index
    if n > 1:
        inner = part_of_row[1:] == part_of_row[:-1]
        a, b = row_ell_len[:-1], row_ell_len[1:]
        _req((a[inner] >= b[inner]).all(), "ELL counts increase inside a partition")
        tie = inner & (a == b)
        _req((perm[:-1][tie] < perm[1:][tie]).all(), "unstable tie order inside a partition")

    # exact content: union == P A P^T
    B = Bperm if Bperm is not None else permute(A, perm)
    order = np.lexsort((col, row))
    row, col, val = row[order], col[order], val[order]
    Brows = np.repeat(np.arange(n), np.diff(B.row_ptr))
    _req(row.size == B.nnz, f"entry count {row.size} != nnz {B.nnz}")
    _req(np.array_equal(row, Brows) and np.array_equal(col, B.col.astype(np.int64)),
         "stored pattern differs from P A P^T")
    want = B.val.astype(value_dtype)
    _req(np.array_equal(np.ascontiguousarray(val).view(np.uint8),
                        np.ascontiguousarray(want).view(np.uint8)),
         "stored values differ from P A P^T bit for bit")
    _req(np.array_equal(row_ell_len + row_er_len, np.diff(B.row_ptr)), "row lengths")

    nnz_er = int((~in_ell).sum())
    return {
        "nnz": int(B.nnz), "nnz_ell": int(in_ell.sum()), "nnz_er": nnz_er,
        "ell_slots": int((meta[:, 1] * 64 * kc).sum()), "er_slots": int((meta[:, 3] * 64).sum()),
        "er_fraction": nnz_er / max(1, B.nnz), "nparts": nparts,
    }
