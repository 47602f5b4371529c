"""The O3 structural checker accepts a hand-built EHYB encoding and rejects
encodings with planted mistakes (mistakes planted in checker inputs, CPU only).

Hand-built example (4x4, two partitions {0,1} and {2,3}, one lane per row,
two entries per lane per step):

    A = [[1 2 . 3]     row 0: ELL (0,0)=1 (0,1)=2, residual (0,3)=3
         [4 5 . .]     row 1: ELL (1,0)=4 (1,1)=5
         [. . 6 7]     row 2: ELL (2,2)=6 (2,3)=7
         [8 . 9 10]]   row 3: ELL (3,2)=9 (3,3)=10, residual (3,0)=8
"""
import numpy as np
import pytest

import matgen
from oracle.structure import PlanError, check_plan, layout_spmv


def _tiny():
    d = np.array([[1, 2, 0, 3], [4, 5, 0, 0], [0, 0, 6, 7], [8, 0, 9, 10]], dtype=np.float64)
    A = matgen.from_dense(d)
    ell_val = np.zeros(256)
    ell_col = np.zeros(256, dtype=np.uint16)
    for slot, v, c in [(0, 1, 0), (1, 2, 1), (2, 4, 0), (3, 5, 1),
                       (128, 6, 0), (129, 7, 1), (130, 9, 0), (131, 10, 1)]:
        ell_val[slot], ell_col[slot] = v, c
    # residual rows: partition 0 -> local row 0; partition 1 -> local row 1
    er_val = np.zeros(128)
    er_col = np.zeros(128, dtype=np.int32)
    er_val[0], er_col[0] = 3, 3
    er_val[64], er_col[64] = 8, 0
    er_row = np.full((2, 64), 0xFFFF, dtype=np.uint16)
    er_row[0, 0], er_row[1, 0] = 0, 1
    view = dict(n=4, nparts=2, L=1, kc=2, perm=np.arange(4), part_start=np.array([0, 2, 4]),
                slice_start=np.array([0, 1, 2]), er_slice_start=np.array([0, 1, 2]),
                ell_free=np.array([0, 0]), halo_start=np.array([0, 0, 0]),
                halo_idx=np.zeros(0, dtype=np.int32),
                ell_meta=np.array([[0, 2, 0b01, 0], [128, 2, 0b10, 0]], dtype=np.uint32),
                er_meta=np.array([[0, 1], [64, 1]], dtype=np.uint32), er_row=er_row,
                ell_val=ell_val, ell_col=ell_col, er_val=er_val, er_col=er_col,
                row_ell_len=np.array([2, 2, 2, 2]), row_er_len=np.array([1, 0, 0, 1]))
    return A, d, view


def test_hand_built_plan_passes():
    A, d, view = _tiny()
    st = check_plan(A, view)
    assert st["nnz_ell"] == 8 and st["nnz_er"] == 2 and st["nparts"] == 2
    x = np.array([1.0, -2.0, 0.5, 3.0])
    assert np.array_equal(layout_spmv(view, x), d @ x)


@pytest.mark.parametrize("mutate,msg", [
    (lambda v: v["ell_val"].__setitem__(1, 2.5), "values differ"),
    (lambda v: v["ell_val"].__setitem__(7, 1.0), "padding"),
    (lambda v: v["ell_val"].__setitem__(7, -0.0), "padding"),
    (lambda v: v["ell_col"].__setitem__(1, 3), "outside"),
    (lambda v: v["er_col"].__setitem__(64, 1), "pattern differs"),
    (lambda v: v["perm"].__setitem__(slice(0, 2), [1, 0]), ""),
    (lambda v: v["row_er_len"].__setitem__(0, 0), ""),
    (lambda v: v["ell_meta"].__setitem__((1, 0), 0), "overlapping"),
    (lambda v: v["ell_meta"].__setitem__((0, 2), 0b10), "mask"),
    (lambda v: v["ell_meta"].__setitem__((0, 2), 0), "queue order"),
    (lambda v: v["ell_free"].__setitem__(0, 1), "queue order"),
    (lambda v: v["er_row"].__setitem__((1, 0), 0), ""),
    (lambda v: v["er_meta"].__setitem__((1, 1), 2), ""),
    (lambda v: v["part_start"].__setitem__(1, 3), ""),
])
def test_planted_mistakes_are_caught(mutate, msg):
    A, _, view = _tiny()
    mutate(view)
    with pytest.raises((PlanError, IndexError, ValueError)) as e:
        check_plan(A, view)
    assert msg in str(e.value)


def test_intra_partition_entry_in_residual_is_caught():
    """Move ELL entry (1,0) into the residual part: same content, wrong class."""
    A, _, view = _tiny()
    view["ell_val"][2], view["ell_val"][3] = 5, 0      # row 1 keeps only (1,1) in ELL
    view["ell_col"][2], view["ell_col"][3] = 1, 0
    view["row_ell_len"][1] = 1
    view["row_er_len"][1] = 1
    view["er_row"][0, 1] = 1                            # residual slice 0: rows 0, 1
    view["er_val"][1], view["er_col"][1] = 4, 0
    view["ell_meta"][0, 2] = 0b11
    with pytest.raises(PlanError, match="intra-partition"):
        check_plan(A, view)
    # a width cap of 1 would need every ELL row to respect it, which rows 0, 2, 3 do not
    with pytest.raises(PlanError):
        check_plan(A, view, width_cap=1)


def _tail():
    """One partition of three rows with 3, 2 and 1 entries, one lane per row,
    two entries per full step: width 3 = one full step (slots 0..127, lane r
    at 2r, 2r+1) and one single-entry step (slots 128..191, lane r at 128+r)."""
    d = np.array([[1, 2, 3], [4, 5, 0], [0, 0, 6]], dtype=np.float64)
    A = matgen.from_dense(d)
    ell_val = np.zeros(192)
    ell_col = np.zeros(192, dtype=np.uint16)
    for slot, v, c in [(0, 1, 0), (1, 2, 1), (128, 3, 2), (2, 4, 0), (3, 5, 1), (4, 6, 2)]:
        ell_val[slot], ell_col[slot] = v, c
    er_row = np.zeros((0, 64), dtype=np.uint16)
    view = dict(n=3, nparts=1, L=1, kc=2, perm=np.arange(3), part_start=np.array([0, 3]),
                slice_start=np.array([0, 1]), er_slice_start=np.array([0, 0]),
                ell_free=np.array([1]), halo_start=np.array([0, 0]), halo_idx=np.zeros(0, dtype=np.int32),
                ell_meta=np.array([[0, 3, 0, 0]], dtype=np.uint32),
                er_meta=np.zeros((0, 2), dtype=np.uint32), er_row=er_row,
                ell_val=ell_val, ell_col=ell_col, er_val=np.zeros(0), er_col=np.zeros(0, dtype=np.int32),
                row_ell_len=np.array([3, 2, 1]), row_er_len=np.array([0, 0, 0]))
    return A, d, view


def test_single_entry_steps_after_full_steps():
    A, d, view = _tail()
    st = check_plan(A, view)
    assert st["ell_slots"] == 192 and st["nnz_ell"] == 6
    x = np.array([1.0, -2.0, 0.5])
    assert np.array_equal(layout_spmv(view, x), d @ x)


@pytest.mark.parametrize("mutate", [
    lambda v: v["ell_meta"].__setitem__((0, 1), 4),                  # wider than the longest row needs
    lambda v: v["ell_meta"].__setitem__((0, 1), 2),                  # too narrow for row 0
    lambda v: (v["ell_val"].__setitem__(128, 0.0), v["ell_val"].__setitem__(2 * 0 + 2, 3.0)),
    lambda v: (v["ell_val"].__setitem__(128, 0.0), v["ell_val"].__setitem__(129, 3.0),
               v["ell_col"].__setitem__(129, 2)),                    # entry 2 of row 0 in lane 1
])
def test_single_entry_step_mistakes_are_caught(mutate):
    A, _, view = _tail()
    mutate(view)
    with pytest.raises((PlanError, IndexError, ValueError)):
        check_plan(A, view)


def test_lds_budget_and_16bit_limit():
    A, _, view = _tiny()
    with pytest.raises(PlanError, match="on-chip"):
        check_plan(A, view, x_bytes=8, lds_budget=8)


def _wide_view():
    """A power-law plan with the paper's split (no halo): hub rows have more
    than 32 residual entries and get wide residual slices."""
    from paper_2204_06666_amd import Plan
    A = matgen.powerlaw(3000, exponent=2.3, mean_deg=12, seed=9)
    P = Plan(A, slice_rows=400, halo_rows=-1)
    arr = P.arrays()
    view = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in arr.items()}
    view["er_meta"] = view["er_meta"].reshape(-1, 2)
    view["er_row"] = view["er_row"].reshape(-1, 64 // view["L"])
    return A, view


def test_wide_residual_slices_pass_and_interpret():
    A, view = _wide_view()
    st = check_plan(A, view)
    assert st["n_er_wide"] > 0
    x = matgen.uniform_vector(A.n_rows, 4)
    perm = np.asarray(view["perm"])
    import oracle
    yp = layout_spmv(view, x[perm])
    y = np.empty_like(yp)
    y[perm] = yp
    oracle.assert_close(y, oracle.spmv(A, x), oracle.abs_scale(A, x), 1e-12, "wide slices")


def test_wide_slice_mistakes_are_caught():
    A, view = _wide_view()
    wide = np.nonzero(view["er_meta"][:, 1] & (1 << 31))[0]
    normal = np.nonzero((view["er_meta"][:, 1] & (1 << 31)) == 0)[0]
    v1 = {k: (a.copy() if isinstance(a, np.ndarray) else a) for k, a in view.items()}
    v1["er_meta"][wide[0], 1] &= np.uint32(0x7FFFFFFF)  # a long row left to one lane group
    with pytest.raises(PlanError):
        check_plan(A, v1)
    v2 = {k: (a.copy() if isinstance(a, np.ndarray) else a) for k, a in view.items()}
    v2["er_meta"][normal[-1], 1] |= np.uint32(1 << 31)  # a short-row slice flagged wide
    with pytest.raises(PlanError):
        check_plan(A, v2)
