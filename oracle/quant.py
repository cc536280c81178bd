"""Low-precision storage formats of the precision mode (TEST INFRASTRUCTURE ONLY).

Written from the format definitions, independently of the GPU library:
* BF16: the top 16 bits of the FP32 pattern after round-to-nearest-even.
* FP16: IEEE binary16, round-to-nearest-even, saturated to +-65504.
* FP8: OCP E4M3 ("FN": bias 7, 3 mantissa bits, no infinities, 0x7F/0xFF
  NaN, largest finite 448), round-to-nearest-even, saturated to +-448, with
  one FP32 scale per vector s = max_j |x_j| / 448 (1 for the zero vector);
  the stored code is E4M3(x_j / s) and the represented value s * E4M3 value.
"""
from __future__ import annotations

import numpy as np


def bf16_bits(x) -> np.ndarray:
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = u + 0x7FFF + ((u >> 16) & 1)
    return (u >> 16).astype(np.uint16)


def bf16_value(bits) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint32) << 16).view(np.float32)


def f16_bits(x) -> np.ndarray:
    x = np.clip(np.asarray(x, dtype=np.float32), -65504.0, 65504.0)
    return x.astype(np.float16).view(np.uint16)


def e4m3_value(code) -> np.ndarray:
    """Decode E4M3 codes (NaN codes decode to NaN)."""
    c = np.asarray(code, dtype=np.int64)
    s = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    v = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1 + m / 8.0) * 2.0 ** (e - 7))
    v = np.where((c & 0x7F) == 0x7F, np.nan, v)
    return (s * v).astype(np.float64)


_FINITE = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.int64)
_FVAL = e4m3_value(_FINITE)


def e4m3_code(x) -> np.ndarray:
    """Round each FP32 value to the nearest finite E4M3 value, ties to the
    even code (even mantissa), saturating beyond +-448."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    pos = np.abs(x)
    pcodes = _FINITE[_FINITE < 0x80]          # 0x00 .. 0x7E, increasing values
    pvals = _FVAL[_FINITE < 0x80]
    i = np.searchsorted(pvals, pos, side="left")
    i = np.clip(i, 1, len(pvals) - 1)
    lo, hi = pvals[i - 1], pvals[i]
    take_hi = (pos - lo > hi - pos) | ((pos - lo == hi - pos) & ((pcodes[i] & 1) == 0))
    c = np.where(take_hi, pcodes[i], pcodes[i - 1])
    c = np.where(pos >= pvals[-1], 0x7E, c)
    c = np.where(pos <= 0, 0, c)
    neg = (x < 0) & (c != 0)
    return np.where(neg, c | 0x80, c).astype(np.uint8)


def fp8_scale(rows) -> np.ndarray:
    rows = np.asarray(rows, dtype=np.float32)
    amax = np.max(np.abs(rows), axis=1)
    return np.where(amax > 0, (amax / np.float32(448.0)).astype(np.float32), np.float32(1.0))


def fp8_rows(rows):
    """Per-vector scale and codes, codes = E4M3(x_j / s) with the FP32 quotient."""
    rows = np.asarray(rows, dtype=np.float32)
    s = fp8_scale(rows)
    q = (rows / s[:, None]).astype(np.float32)
    return s, e4m3_code(q)


def pad_cols(a, dpad):
    out = np.zeros((a.shape[0], dpad), dtype=a.dtype)
    out[:, :a.shape[1]] = a
    return out
