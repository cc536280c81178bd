"""Pins for the precision-mode storage formats (oracle/quant.py) against
library conversions and the format definitions."""
import numpy as np
import pytest
import torch

from oracle import quant


def _edge_floats():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-6, 6, size=4000),
                        [0.0, -0.0, 1.0, -1.0, 3.1415927, 65504.0, 65519.0, 1e-40, -1e-40,
                         448.0, 449.0, 1e6, -1e6, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -11]])
    return v.astype(np.float32)


def test_bf16_matches_torch():
    v = _edge_floats()
    ref = torch.from_numpy(v).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(quant.bf16_bits(v), ref)


def test_bf16_ties_to_even():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: rounds to the even 1.0
    assert quant.bf16_bits(np.float32(1 + 2 ** -8)) == 0x3F80
    # 1 + 3*2^-8 halfway between 1+2^-7 (odd) and 1+2^-6 (even): rounds up
    assert quant.bf16_bits(np.float32(1 + 3 * 2 ** -8)) == 0x3F82


def test_f16_matches_numpy_and_saturates():
    v = np.array([1.0, 0.1, -2.5, 1e-8, 65504.0, 70000.0, -1e9], np.float32)
    b = quant.f16_bits(v)
    assert np.array_equal(b[:4], v[:4].astype(np.float16).view(np.uint16))
    assert b[5] == np.float16(65504).view(np.uint16) and b[6] == np.float16(-65504).view(np.uint16)


def test_e4m3_decode_encode_identity_all_finite_codes():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F and c != 0x80], np.uint8)
    vals = quant.e4m3_value(codes).astype(np.float32)
    assert np.array_equal(quant.e4m3_code(vals), codes)
    assert quant.e4m3_value(0x7E) == 448.0 and quant.e4m3_value(0x01) == 2.0 ** -9
    assert quant.e4m3_value(0x08) == 2.0 ** -6


def test_e4m3_ties_and_saturation():
    # between 1.0 (0x38) and 1.125 (0x39): midpoint 1.0625 -> even code 0x38
    assert quant.e4m3_code(np.float32(1.0625)) == 0x38
    # between 1.125 (0x39) and 1.25 (0x3A): midpoint 1.1875 -> 0x3A
    assert quant.e4m3_code(np.float32(1.1875)) == 0x3A
    # subnormal midpoint 1.5 * 2^-9 between 0x01 and 0x02 -> 0x02
    assert quant.e4m3_code(np.float32(1.5 * 2 ** -9)) == 0x02
    for v in (448.0, 460.0, 470.0, 1e6):
        assert quant.e4m3_code(np.float32(v)) == 0x7E
        assert quant.e4m3_code(np.float32(-v)) == 0xFE


def test_e4m3_matches_torch_in_range():
    v = _edge_floats()
    v = v[np.abs(v) < 448.0]
    ref = torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = quant.e4m3_code(v)
    # torch keeps the sign of a value that rounds to zero; the format has a
    # single zero here (code 0)
    ref = np.where((ref & 0x7F) == 0, 0, ref)
    assert np.array_equal(got, ref)


def test_fp8_rows_scale():
    rows = np.array([[1.0, -2.0, 0.5], [0.0, 0.0, 0.0], [448.0, 1.0, -896.0]], np.float32)
    s, c = quant.fp8_rows(rows)
    assert s[0] == np.float32(2.0) / np.float32(448.0) and s[1] == 1.0
    assert np.all(c[1] == 0)
    # the largest magnitude of every nonzero row maps to +-448
    assert quant.e4m3_value(c[0][1]) == -448.0 and quant.e4m3_value(c[2][2]) == -448.0
