"""O3: structural checker of an EHYB encoding (test infrastructure only).

An independent reader of the EHYB arrays.  It re-derives, from the layout
rules alone, which stored slot holds which matrix entry, and then checks the
properties the paper fixes for the format:

* the row permutation is a bijection, and rows of one partition are contiguous
  (Section 3.1: partitions own blocks of rows; Alg. 1 builds the reorder table);
* every partition's slice of x fits the on-chip cache and its local column
  indices fit 16 bits (Section 3.3, Eq. 1-2; Section 3.4, compact index);
* every stored entry of the ELL part has its column inside the row's own
  partition or in the partition's halo (the out-of-partition x entries it
  caches next to its x-slice), and (with no width cap) every such entry is in
  the ELL part, every other entry in the residual ("extra rows") part
  (Section 3.1-3.2, Alg. 1 classification);
* within a partition, rows are ordered by non-increasing ELL entry count
  (Section 3.2, post-partitioning reordering), ties broken by original index;
* padding slots hold +0.0 and a valid column;
* the union of both parts is exactly P A P^T, values bit for bit (the reorder
  of Alg. 2 moves values without touching them).

Layout rules being checked (row-slice = C = 64 / L rows, one 64-lane
wavefront per row-slice, L lanes per row).  ELL part: partition p's rows, in order, cut into row-slices; row r of
an ELL slice with index j is local row j*C + r.  Residual part: the rows
of partition p that have residual entries, by non-increasing residual count
(ties by local row), cut into row-slices; row r of residual slice e is local
row er_row[e, r] (0xFFFF: none).  When C > 1, every residual row with more
than 32*L residual entries comes first, in a "wide" slice of its own (bit 31
of its step count, row at r = 0) laid out as if L were 64.

An ELL slice of width W (entries per lane) has F = W // kc full steps of kc
consecutive entries per lane, then W % kc single-entry steps; a residual
slice of S steps has F = S steps of one entry per lane.  Entry k (ascending
column) of row r of a slice with slot offset `off` lives at

    k <  F*L*KC:  t = k // (L*KC), u = (k // KC) % L, c = k % KC,
                  slot = off + (t*64 + r*L + u)*KC + c,
    k >= F*L*KC:  k1 = k - F*L*KC, slot = off + F*64*KC + (k1 // L)*64 + r*L + k1 % L,

with KC = kc in the ELL part and KC = 1 in the residual part.  A slice holds
64*W (ELL) or 64*S (residual) slots, and W is the least width that holds the
slice's longest row: W = (m // (L*kc))*kc + ceil((m mod L*kc) / L).

ELL columns are 16-bit indices into the partition's LDS vector: below the
partition size an x-slice element, otherwise halo element
halo_idx[halo_start[p] + c - size].

``view`` is a mapping with the keys: n, nparts, L, kc, perm, part_start,
halo_start, halo_idx, slice_start, er_slice_start, ell_free, ell_meta (uint32 [nslices, 4]: offset,
width | slice index << 16, residual-row mask low/high; slices without residual
rows first), er_meta (uint32 [ner_slices, 2]: offset, steps | wide << 31),
er_row (uint16 [ner_slices, C]), ell_val, ell_col (uint16), er_val, er_col
(int32), row_ell_len, row_er_len.
"""
from __future__ import annotations

import numpy as np


class PlanError(AssertionError):
    pass


def _req(cond, msg):
    if not cond:
        raise PlanError(msg)


WIDE = 1 << 31        # step-count flag of a wide residual slice
WIDE_STEPS = 32      # a residual row longer than WIDE_STEPS * L entries is wide


def _slice_rows(view, which: str):
    """Per slice: (slot offset, lane width, partition, rows[C], wide): the lane
    width is the ELL width W or the residual step count S (the slots of one
    lane), rows the permuted row of each slice row or -1, wide the wide-slice
    flag."""
    L = int(view["L"])
    C = 64 // L
    part_start = np.asarray(view["part_start"], dtype=np.int64)
    nparts = len(part_start) - 1
    if which == "ell":
        meta = np.asarray(view["ell_meta"], dtype=np.int64).reshape(-1, 4)
        starts = np.asarray(view["slice_start"], dtype=np.int64)
    else:
        meta = np.asarray(view["er_meta"], dtype=np.int64).reshape(-1, 2)
        starts = np.asarray(view["er_slice_start"], dtype=np.int64)
    ns = meta.shape[0]
    _req(starts.shape == (nparts + 1,) and starts[0] == 0 and starts[-1] == ns,
         f"{which} slice bounds do not cover its metadata")
    _req((np.diff(starts) >= 0).all(), f"{which} slice bounds decrease")
    part = np.repeat(np.arange(nparts), np.diff(starts))
    if which == "ell":
        width = meta[:, 1] & 0xFFFF
        j = meta[:, 1] >> 16
        local = j[:, None] * C + np.arange(C)[None, :]
        size = (part_start[part + 1] - part_start[part])[:, None]
        rows = np.where(local < size, part_start[part][:, None] + local, -1)
        wide = np.zeros(ns, dtype=bool)
    else:
        width = meta[:, 1] & (WIDE - 1)
        wide = (meta[:, 1] & WIDE) != 0
        er_row = np.asarray(view["er_row"], dtype=np.int64).reshape(ns, C)
        rows = np.where(er_row != 0xFFFF, part_start[part][:, None] + er_row, -1)
    return meta[:, 0], width, part, rows, wide


def _slots(view, which: str):
    """Enumerate every slot of one part.

    Returns (slot, row, k, valid, part): the slot index, the permuted row it
    belongs to (-1 for slice rows that hold no row), the entry position within
    the row, whether it holds a real entry, and the slice's partition."""
    L = int(view["L"])
    kc = int(view["kc"]) if which == "ell" else 1
    off, width, part_of_slice, rows, wide = _slice_rows(view, which)
    rowlen = np.asarray(view["row_ell_len"] if which == "ell" else view["row_er_len"],
                        dtype=np.int64)
    nslices = off.shape[0]
    per = width * 64
    total = int(per.sum())
    s_of = np.repeat(np.arange(nslices), per)
    o = np.arange(total) - np.repeat(np.cumsum(per) - per, per)
    full = (width // kc)[s_of]           # steps of kc entries per lane
    Ls = np.where(wide[s_of], 64, L)     # lanes per row of each slot's slice
    in_full = o < full * 64 * kc
    o1 = o - full * 64 * kc              # position among the single-entry steps
    lane = np.where(in_full, (o // kc) % 64, o1 % 64)
    r = lane // Ls
    u = lane % Ls
    k = np.where(in_full, ((o // (64 * kc)) * Ls + u) * kc + o % kc, full * Ls * kc + (o1 // 64) * Ls + u)
    row = rows[s_of, r] if total else np.zeros(0, dtype=np.int64)
    exists = row >= 0
    valid = exists.copy()
    valid[exists] = k[exists] < rowlen[row[exists]]
    slot = off[s_of] + o
    return slot, row, k, valid, part_of_slice[s_of]


def _ell_global(view, local, part):
    """Permuted global column of ELL local columns: below the partition size
    an x-slice element, otherwise a halo element."""
    part_start = np.asarray(view["part_start"], dtype=np.int64)
    halo_start = np.asarray(view["halo_start"], dtype=np.int64)
    halo_idx = np.asarray(view["halo_idx"], dtype=np.int64)
    size = part_start[part + 1] - part_start[part]
    own = local < size
    out = np.empty_like(local)
    out[own] = part_start[part[own]] + local[own]
    k = halo_start[part[~own]] + local[~own] - size[~own]
    _req((k < halo_start[part[~own] + 1]).all(), "ELL column past the end of its halo")
    out[~own] = halo_idx[k]
    return out


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
            col = _ell_global(view, col, part[valid])
        out.append((row[valid], col, vals[sv], np.full(sv.size, which == "ell")))
    return tuple(np.concatenate([o[i] for o in out]) for i in range(4))


def stored_values_f64(view, vals) -> np.ndarray:
    """Stored values as float64 (bfloat16 plans keep bit patterns; value
    types 2 and 4 store bfloat16, 1 and 3 binary32, 0 binary64)."""
    if int(view.get("value_dtype", 0)) in (2, 4):
        from .precision import bf16_bits_to_f64
        return bf16_bits_to_f64(vals)
    return np.asarray(vals).astype(np.float64)


def layout_spmv(view, xp: np.ndarray) -> np.ndarray:
    """Execute the EHYB arrays as laid out (a sequential format interpreter):
    y_p = sum over real slots of the row of val * xp[col], in permuted space."""
    row, col, val, _ = layout_entries(view)
    n = int(view["n"])
    return np.bincount(row, weights=stored_values_f64(view, val) * xp[col], minlength=n)


def check_plan(A, view, x_bytes: int = 8, lds_budget: int = 160 * 1024, width_cap: int = 0,
               value_dtype=np.float64, Bperm=None, acc_bytes: int | None = None) -> dict:
    """Check every structural property of an EHYB encoding of ``A``.

    ``value_dtype`` is the storage type of values (float64 plans must reproduce
    A's bits; float32 and "bf16" plans must reproduce A's values rounded to
    nearest-even in that type).  ``acc_bytes`` is the size of a residual
    accumulator in LDS (default x_bytes; 8 for binary64 accumulation).  ``Bperm`` may pass a precomputed P A P^T.  Returns statistics."""
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
    # halo: ascending permuted indices outside the partition
    halo_start = np.asarray(view["halo_start"], dtype=np.int64)
    halo_idx = np.asarray(view["halo_idx"], dtype=np.int64)
    _req(halo_start.shape == (nparts + 1,) and (nparts == 0 or halo_start[0] == 0)
         and (nparts == 0 or halo_start[-1] == halo_idx.size) and (np.diff(halo_start) >= 0).all(),
         "halo bounds")
    hsz = np.diff(halo_start)
    hpart = np.repeat(np.arange(nparts), hsz)
    _req(((halo_idx >= 0) & (halo_idx < n)).all(), "halo index out of range")
    _req(((halo_idx < part_start[hpart]) | (halo_idx >= part_start[hpart + 1])).all(),
         "halo entry inside its own partition")
    inner = hpart[1:] == hpart[:-1]
    _req((np.diff(halo_idx)[inner] > 0).all(), "halo not strictly ascending")
    _req((sizes + hsz <= 65535).all(), "LDS vector larger than a 16-bit local index allows")
    has_er = int(np.asarray(view["er_meta"]).size) > 0
    ab = x_bytes if acc_bytes is None else acc_bytes       # bytes of one residual accumulator
    xs_bytes = (sizes.max(initial=0) + hsz.max(initial=0)) * x_bytes
    lds = (-(-xs_bytes // ab) * ab + sizes.max(initial=0) * ab) if has_er else xs_bytes
    _req(lds <= lds_budget, "x-slice, halo and residual accumulators exceed the on-chip budget")

    L = int(view["L"])
    _req(L in (1, 2, 4, 8, 16, 32, 64), "lanes per row must divide 64")
    C = 64 // L
    slice_start = np.asarray(view["slice_start"], dtype=np.int64)
    _req(np.array_equal(np.diff(slice_start), -(-sizes // C)), "ELL slices per partition")
    # ELL slices in queue order: the slices without residual rows (ascending),
    # then the others (ascending); ell_free counts the first group
    ell_meta = np.asarray(view["ell_meta"], dtype=np.int64).reshape(-1, 4)
    ell_free = np.asarray(view["ell_free"], dtype=np.int64)
    _req(ell_free.shape == (nparts,), "ell_free length")
    jj = ell_meta[:, 1] >> 16
    dep = (ell_meta[:, 2] | ell_meta[:, 3]) != 0
    for p in range(nparts):
        a, b = slice_start[p], slice_start[p + 1]
        _req(np.array_equal(np.sort(jj[a:b]), np.arange(b - a)), "ELL slice indices are not a permutation")
        f = int(ell_free[p])
        _req(0 <= f <= b - a and not dep[a:a + f].any() and dep[a + f:b].all(),
             "ELL slices not in queue order (free slices first)")
        _req((np.diff(jj[a:a + f]) > 0).all() and (np.diff(jj[a + f:b]) > 0).all(),
             "ELL slices within a queue group are not ascending")

    kc = int(view["kc"])
    ell_val = np.asarray(view["ell_val"])
    er_val = np.asarray(view["er_val"])
    ell_col = np.asarray(view["ell_col"])
    er_col = np.asarray(view["er_col"])
    _req(ell_col.dtype == np.uint16, "ELL columns must be 16-bit")
    row_ell_len = np.asarray(view["row_ell_len"], dtype=np.int64)
    row_er_len = np.asarray(view["row_er_len"], dtype=np.int64)
    part_of_row = np.repeat(np.arange(nparts), sizes)

    # residual rows: exactly the rows with residual entries, each once, in
    # non-increasing residual count, ties by local row, padding at the end
    er_row = np.asarray(view["er_row"], dtype=np.int64).reshape(-1, C)
    er_start = np.asarray(view["er_slice_start"], dtype=np.int64)
    er_wide = (np.asarray(view["er_meta"], dtype=np.int64).reshape(-1, 2)[:, 1] & WIDE) != 0
    for p in range(nparts):
        a, b = er_start[p], er_start[p + 1]
        w = er_wide[a:b]
        nw = int(w.sum())
        _req(not w[nw:].any(), "wide residual slices are not first")
        _req(nw == 0 or C > 1, "wide residual slice with one row per slice")
        _req((er_row[a:a + nw, 0] != 0xFFFF).all() and (er_row[a:a + nw, 1:] == 0xFFFF).all(),
             "a wide residual slice must hold exactly one row, at r = 0")
        rows_n = er_row[a + nw:b].reshape(-1)
        real_n = rows_n[rows_n != 0xFFFF]
        _req(np.array_equal(rows_n[:real_n.size], real_n), "residual padding rows before real rows")
        real = np.concatenate([er_row[a:a + nw, 0], real_n])
        want = np.nonzero(row_er_len[part_start[p]:part_start[p + 1]] > 0)[0]
        _req(real.size == want.size and np.array_equal(np.sort(real), want),
             "residual rows are not exactly the rows with residual entries")
        lens_p = row_er_len[part_start[p] + real]
        long_rows = int((lens_p > WIDE_STEPS * L).sum()) if C > 1 else 0
        _req(nw == long_rows and (lens_p[:nw] > WIDE_STEPS * L).all(),
             "wide residual slices are not exactly the rows longer than 32 * L entries")
        _req(rows_n.size == -(-(want.size - nw) // C) * C, "residual slices per partition")
        cnt = row_er_len[part_start[p] + real]
        _req((np.diff(cnt) <= 0).all(), "residual rows not in non-increasing residual count")
        tie = np.diff(cnt) == 0
        _req((np.diff(real)[tie] > 0).all(), "residual rows: unstable tie order")

    for which, arr in (("ell", ell_val), ("er", er_val)):
        off, width, part_of_slice, rows, wide = _slice_rows(view, which)
        end = off + width * 64
        _req((end <= arr.size).all(), "slot range past the end of its array")
        o = np.argsort(off, kind="stable")
        nz = width[o] > 0
        _req((off[o][nz][1:] >= end[o][nz][:-1]).all(), "overlapping slot ranges")
        # minimal widths: each slice is as wide as its longest row needs
        lens = row_ell_len if which == "ell" else row_er_len
        rl = np.where(rows >= 0, lens[np.maximum(rows, 0)], 0)
        need = rl.max(axis=1) if rl.size else np.zeros(0, dtype=np.int64)
        if which == "ell":
            fs = need // (L * kc)
            want_w = fs * kc + -(-(need - fs * L * kc) // L)
        else:
            want_w = -(-need // np.where(wide, 64, L))
        _req(np.array_equal(width, want_w), f"{which} slice width is not its longest row")
        if which == "ell":
            meta = np.asarray(view["ell_meta"], dtype=np.uint64).reshape(-1, 4)
            mask = meta[:, 2] | (meta[:, 3] << np.uint64(32))
            has = np.where(rows >= 0, row_er_len[np.maximum(rows, 0)] > 0, False)
            bits = (mask[:, None] >> np.arange(C, dtype=np.uint64)[None, :]) & np.uint64(1)
            _req(np.array_equal(bits.astype(bool), has), "ELL residual-row mask is wrong")
            if C < 64:
                _req(((mask >> np.uint64(C)) == 0).all(), "ELL residual-row mask names a missing row")

    # padding slots
    for which, vals, cols in (("ell", ell_val, ell_col), ("er", er_val, er_col)):
        slot, row, k, valid, part = _slots(view, which)
        pad = slot[~valid]
        bits = np.ascontiguousarray(vals[pad]).view(np.uint8)
        _req(not bits.any(), f"{which} padding slot is not +0.0")
        pc = cols[pad].astype(np.int64)
        if which == "ell":
            ext = sizes + hsz
            _req((pc < ext[part[~valid]]).all(), "ELL padding column outside its LDS vector")
            rv = row[valid]
            _req((cols[slot[valid]].astype(np.int64) < ext[part_of_row[rv]]).all(),
                 "ELL local column outside its LDS vector")
        else:
            _req(((pc >= 0) & (pc < n)).all(), "residual padding column out of range")
            _req((part_of_row[row[valid]] == part[valid]).all(),
                 "residual row outside its slice's partition")

    row, col, val, in_ell = layout_entries(view)
    _req(((col >= 0) & (col < n)).all(), "column out of range")
    rp = part_of_row[row]
    same = rp == part_of_row[col]
    # column cached in the row's halo?
    if halo_idx.size:
        key_h = hpart.astype(np.int64) * (n + 1) + halo_idx
        key_e = rp.astype(np.int64) * (n + 1) + col
        pos = np.clip(np.searchsorted(key_h, key_e), 0, key_h.size - 1)
        cached = key_h[pos] == key_e
    else:
        cached = np.zeros(row.size, dtype=bool)
    served = same | cached
    _req(served[in_ell].all(), "ELL entry whose column is neither in the partition nor in its halo")
    if width_cap == 0:
        _req((~served[~in_ell]).all(), "intra-partition entry left in the residual part")
    else:
        _req((row_ell_len <= width_cap).all(), "ELL row longer than the width cap")
        spill = ~in_ell & served
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
    if isinstance(value_dtype, str) and value_dtype == "bf16":
        from .precision import to_bf16_bits
        want = to_bf16_bits(B.val)
    else:
        want = B.val.astype(value_dtype)
    _req(np.array_equal(np.ascontiguousarray(val).view(np.uint8),
                        np.ascontiguousarray(want).view(np.uint8)),
         "stored values differ from P A P^T bit for bit")
    _req(np.array_equal(row_ell_len + row_er_len, np.diff(B.row_ptr)), "row lengths")

    nnz_er = int((~in_ell).sum())
    return {
        "nnz": int(B.nnz), "nnz_ell": int(in_ell.sum()), "nnz_er": nnz_er,
        "nnz_halo": int((in_ell & ~same).sum()), "n_halo": int(halo_idx.size),
        "ell_slots": int((np.asarray(view["ell_meta"], dtype=np.int64).reshape(-1, 4)[:, 1] & 0xFFFF).sum() * 64),
        "er_slots": int((np.asarray(view["er_meta"], dtype=np.int64).reshape(-1, 2)[:, 1] & (WIDE - 1)).sum() * 64),
        "n_er_wide": int(er_wide.sum()),
        "er_fraction": nnz_er / max(1, B.nnz), "nparts": nparts,
    }
