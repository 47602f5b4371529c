"""Pins of the reduced-precision oracle helpers (bfloat16 / binary32 rounding)."""
import numpy as np
import pytest

import matgen
from oracle.precision import bf16_bits_to_f64, gamma32, quantize, to_bf16_bits


def _bit_trick(f32: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even binary32 -> bfloat16 on the bit pattern (finite inputs)."""
    b = f32.view(np.uint32).astype(np.uint64)
    return ((b + 0x7FFF + ((b >> 16) & 1)) >> 16).astype(np.uint16)


def test_hand_values():
    one = 1.0
    cases = {
        one: 0x3F80,
        one + 2.0 ** -8: 0x3F80,            # tie -> even (mantissa 0)
        one + 3 * 2.0 ** -8: 0x3F82,        # tie between 1+2^-7 and 1+2^-6 -> even
        one + 2.0 ** -8 + 2.0 ** -30: 0x3F81,  # just above the tie: rounding via binary32 would give 0x3F80
        -2.0: 0xC000,
        0.0: 0x0000,
        3.0e38: 0x7F62,
        3.4e38: 0x7F80,                     # beyond the largest bfloat16 -> inf
        2.0 ** -133: 0x0001,                # smallest subnormal
    }
    for v, want in cases.items():
        assert int(to_bf16_bits(np.array([v]))[0]) == want, (v, hex(int(to_bf16_bits(np.array([v]))[0])))
    assert int(to_bf16_bits(np.array([-0.0]))[0]) == 0x8000


def test_agrees_with_bit_trick_on_binary32_values():
    g = matgen.rng(5)
    f = (g.standard_normal(200000) * 2.0 ** g.integers(-60, 60, 200000)).astype(np.float32)
    # add exact ties: low 16 bits = 0x8000
    t = (f.view(np.uint32) & np.uint32(0xFFFF0000)) | np.uint32(0x8000)
    f = np.concatenate([f, t.view(np.float32)])
    assert np.array_equal(to_bf16_bits(f.astype(np.float64)), _bit_trick(f))


def test_roundtrip_and_error_bound():
    g = matgen.rng(6)
    v = g.uniform(-1, 1, 100000)
    q = quantize(v, "bf16")
    assert np.all(np.abs(q - v) <= 2.0 ** -8 * np.abs(v))          # half a spacing of 2^-7 relative
    assert np.array_equal(quantize(q, "bf16"), q)                    # idempotent
    assert np.array_equal(bf16_bits_to_f64(to_bf16_bits(q)), q)
    q32 = quantize(v, "f32")
    assert np.all(np.abs(q32 - v) <= 2.0 ** -24 * np.abs(v))


@pytest.mark.parametrize("m", [1, 27, 1000])
def test_gamma32(m):
    u = 2.0 ** -24
    assert gamma32(m) == pytest.approx(m * u / (1 - m * u), rel=1e-15)
