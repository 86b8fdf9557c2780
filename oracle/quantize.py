"""Storage formats of A for the precision forms, written out from their definitions.

TEST INFRASTRUCTURE ONLY (see ``oracle/nsrgs.py``).  Shares no code with the
GPU library's conversion kernels; tests compare the two bit for bit.

The measurement matrix is made in float64 and rounded once to float32
(round-to-nearest-even).  The reduced formats are derived from that float32
matrix, as a one-time conversion of a stored FP32 A would:

* BF16       : bfloat16(a32), round to nearest, ties to even.
* BF16 split : hi = bfloat16(a32), lo = bfloat16(a32 - hi); a32 - hi is exact
               in float32, so hi + lo carries 16 significant bits.
* FP8 e4m3   : OCP 8-bit float E4M3 (1 sign, 4 exponent bits with bias 7,
               3 mantissa bits; no infinities; 0x7F/0xFF are NaN; largest finite
               value 448; subnormals down to 2^-9).  Per row r the scale is
               s_r = max_c |a32_rc| / 448 in float32 (s_r = 1 for an all-zero
               row), and the code is e4m3(a32_rc / s_r) with round to nearest
               even and saturation to +-448.  The value it stands for is
               s_r * e4m3_value, exact in float64.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "to_f32", "bf16_bits", "bf16_value", "bf16_split", "e4m3_table",
    "e4m3_encode", "e4m3_decode", "fp8_rowscaled", "stored_value",
]


def to_f32(a: np.ndarray) -> np.ndarray:
    """float64 -> float32, round to nearest even (IEEE conversion)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def bf16_bits(a32: np.ndarray) -> np.ndarray:
    """bfloat16 codes (uint16) of float32 values, round to nearest even.

    The code is the upper half of the float32 bit pattern after adding
    0x7FFF plus the lowest kept bit (the tie-to-even rule).  NaNs map to a
    quiet NaN with the same sign.
    """
    a32 = np.ascontiguousarray(a32, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) & np.uint64(0xFFFF)
    nan = np.isnan(a32)
    r = np.where(nan, ((u >> np.uint64(16)) & np.uint64(0x8000)) | np.uint64(0x7FC0), r)
    return r.astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    """float32 value of bfloat16 codes (exact)."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32)


def bf16_split(a32: np.ndarray):
    """(hi_bits, lo_bits) with hi = bf16(a), lo = bf16(a - hi)."""
    a32 = np.asarray(a32, dtype=np.float32)
    hi = bf16_bits(a32)
    rem = (a32 - bf16_value(hi)).astype(np.float32)
    lo = bf16_bits(rem)
    return hi, lo


def e4m3_table() -> np.ndarray:
    """float64 value of each of the 256 E4M3 codes (NaN for 0x7F and 0xFF)."""
    vals = np.empty(256, dtype=np.float64)
    for code in range(256):
        s = -1.0 if code & 0x80 else 1.0
        e = (code >> 3) & 0xF
        m = code & 0x7
        if e == 0xF and m == 0x7:
            vals[code] = np.nan
        elif e == 0:
            vals[code] = s * (m / 8.0) * 2.0 ** -6
        else:
            vals[code] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return vals


_TABLE = e4m3_table()
_POS_CODES = np.arange(0, 0x7F)          # 0x00..0x7E: 0 and the positive finite values
_POS_VALS = _TABLE[_POS_CODES]            # increasing


def e4m3_decode(codes: np.ndarray) -> np.ndarray:
    return _TABLE[np.asarray(codes, dtype=np.uint8)]


def e4m3_encode(x32: np.ndarray) -> np.ndarray:
    """E4M3 codes of float32 values: nearest value, ties to the even code,
    magnitudes above 448 saturate to 448, NaN -> 0x7F."""
    x = np.asarray(x32, dtype=np.float32).astype(np.float64)
    mag = np.abs(x)
    sat = np.minimum(mag, 448.0)
    hi_idx = np.searchsorted(_POS_VALS, sat, side="left")       # first value >= sat
    hi_idx = np.clip(hi_idx, 0, len(_POS_VALS) - 1)
    lo_idx = np.clip(hi_idx - 1, 0, len(_POS_VALS) - 1)
    v_hi = _POS_VALS[hi_idx]
    v_lo = _POS_VALS[lo_idx]
    d_hi = v_hi - sat
    d_lo = sat - v_lo
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & ((_POS_CODES[hi_idx] & 1) == 0))
    exact = v_hi == sat
    code = np.where(exact | pick_hi, _POS_CODES[hi_idx], _POS_CODES[lo_idx])
    code = code | np.where(np.signbit(x) & (code != 0), 0x80, 0)
    code = np.where(np.signbit(x) & (code == 0), 0x80, code)   # keep -0
    code = np.where(np.isnan(x), 0x7F, code)
    return code.astype(np.uint8)


def fp8_rowscaled(a32: np.ndarray):
    """(codes uint8 [rows, cols], scales float32 [rows]) per the module rule."""
    a32 = np.asarray(a32, dtype=np.float32)
    amax = np.max(np.abs(a32), axis=1)
    scale = (amax / np.float32(448.0)).astype(np.float32)
    scale = np.where(amax == 0, np.float32(1.0), scale).astype(np.float32)
    q = (a32 / scale[:, None]).astype(np.float32)
    return e4m3_encode(q), scale


def stored_value(a64: np.ndarray, fmt: str):
    """The float64 matrix that a given storage format actually holds.

    fmt in {"f64", "f32", "bf16", "bf16_split", "fp8"}.
    """
    a64 = np.asarray(a64, dtype=np.float64)
    if fmt == "f64":
        return a64.copy()
    a32 = to_f32(a64)
    if fmt == "f32":
        return a32.astype(np.float64)
    if fmt == "bf16":
        return bf16_value(bf16_bits(a32)).astype(np.float64)
    if fmt == "bf16_split":
        hi, lo = bf16_split(a32)
        return bf16_value(hi).astype(np.float64) + bf16_value(lo).astype(np.float64)
    if fmt == "fp8":
        q, s = fp8_rowscaled(a32)
        return s.astype(np.float64)[:, None] * e4m3_decode(q)
    raise ValueError(fmt)
