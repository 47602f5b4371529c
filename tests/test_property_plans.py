"""Property tests (hypothesis): random small sparse square matrices with
empty rows, dense rows, explicit zeros and -0.0, under random preprocessing
parameters.  Every plan must pass the structure checker, decode to P A P^T
bit for bit, and its arrays, executed as laid out, must reproduce the
oracle's product."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import matgen
import oracle
from oracle.structure import check_plan, layout_spmv
from paper_2204_06666_amd import Plan


@st.composite
def matrices(draw):
    n = draw(st.integers(1, 160))
    density = draw(st.sampled_from([0.0, 0.01, 0.05, 0.2, 0.6]))
    seed = draw(st.integers(0, 2**31 - 1))
    empty = draw(st.integers(0, n // 3))
    dense_row = draw(st.booleans())
    zeros = draw(st.integers(0, 5))
    neg = draw(st.booleans())
    return matgen.random_small(n, density, seed, empty_rows=empty, dense_row=dense_row and n > 1,
                               explicit_zeros=zeros, negative_zero=neg)


params = st.fixed_dictionaries({
    "slice_rows": st.sampled_from([0, 1, 7, 32, 64, 100]),
    "rows_per_wave": st.sampled_from([1, 2, 8, 16, 64]),
    "halo_rows": st.sampled_from([-1, 0, 3]),
    "ell_width_cap": st.sampled_from([-1, 0, 1, 4]),
    "partitioner": st.sampled_from([0, 1]),
    "value_dtype": st.sampled_from([0, 1, 2, 3, 4]),
})


@settings(max_examples=300, deadline=None, database=None, suppress_health_check=[HealthCheck.too_slow])
@given(A=matrices(), prm=params)
def test_random_plans_are_valid(A, prm):
    P = Plan(A, **prm)
    stt = P.stats()
    v = P.arrays()
    dt = prm["value_dtype"]
    vt = {0: np.float64, 1: np.float32, 2: "bf16", 3: np.float32, 4: "bf16"}[dt]
    check_plan(A, v, width_cap=stt["ell_width_cap"], value_dtype=vt, x_bytes=8 if dt == 0 else 4,
               acc_bytes=8 if dt in (0, 3, 4) else 4)
    rp, ci, val = P.decode()
    B = oracle.permute(A, v["perm"])
    assert np.array_equal(rp, B.row_ptr) and np.array_equal(ci, B.col)
    if dt == 0:
        assert np.array_equal(val.view(np.uint64), B.val.view(np.uint64))
        x = matgen.uniform_vector(A.n_rows, 5)
        perm = v["perm"]
        oracle.assert_close(layout_spmv(v, x[perm]), oracle.spmv(A, x)[perm], oracle.abs_scale(A, x)[perm],
                            what="layout")
