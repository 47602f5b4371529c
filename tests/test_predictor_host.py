"""Host logic of the parameter predictor: target encoding and the ELL width
quantiles (no GPU)."""
import itertools

import numpy as np

import matgen
from paper_2204_06666_amd.predictor import (ROWS_PER_WAVE, SLICE_ROWS, WIDTH_QUANTILES, decode_output,
                                            encode_target, init_params, lds_max_rows, width_cap)


def test_targets_round_trip_every_grid_point():
    for s, q, r in itertools.product(SLICE_ROWS, WIDTH_QUANTILES, ROWS_PER_WAVE):
        t = encode_target(s, q, r)
        assert np.all((t >= 0) & (t <= 1))
        assert decode_output(t) == (s, q, r)
        assert decode_output(t + 0.08) == (s, q, r)        # nearest point within half a step


def test_decode_clamps():
    assert decode_output(np.array([-5.0, -5.0, -5.0])) == (SLICE_ROWS[0], WIDTH_QUANTILES[0], ROWS_PER_WAVE[0])
    assert decode_output(np.array([5.0, 5.0, 5.0])) == (SLICE_ROWS[-1], WIDTH_QUANTILES[-1], ROWS_PER_WAVE[-1])


def test_width_cap_is_lower_quantile():
    lens = np.array([5, 1, 9, 3, 7, 2, 8, 4, 6, 10])
    assert width_cap(lens, None) == 0
    assert width_cap(lens, 0.90) == 9          # sorted[floor(0.9 * 9)] = sorted[8]
    assert width_cap(lens, 0.75) == 7          # sorted[6]
    assert width_cap(np.zeros(4, int), 0.5) == 1


def test_lds_limit_and_init():
    assert lds_max_rows() == (160 * 1024 - 64) // 8
    p = init_params(1)
    assert p.dtype == np.float32 and p.size == 6467
    assert np.all(p[2048:2112] == 0) and abs(np.std(p[:2048]) - np.sqrt(2 / 32)) < 0.02


def test_tuning_matrices_are_seeded():
    d1, A = matgen.tuning_matrix(3, n_hi=20000)
    d2, B = matgen.tuning_matrix(3, n_hi=20000)
    assert d1 == d2 and np.array_equal(A.col, B.col) and np.array_equal(A.val, B.val)
    assert 10_000 * 0.9 <= A.n_rows <= 20_000 * 1.1
