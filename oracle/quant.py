"""Low-precision copies of A, as plain NumPy (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline
leg may import this.

Not part of the paper: the BF16 / FP8 copies of A that feed the block
products.  Written from the format definitions:
* bfloat16: the top 16 bits of an IEEE binary32, round to nearest even.
* OCP e4m3 ("E4M3FN", OCP 8-bit floating point specification): 1 sign bit,
  4 exponent bits (bias 7), 3 mantissa bits, subnormals with exponent -6, no
  infinities, 0x7F / 0xFF are NaN, largest finite 448.  Conversion rounds to
  nearest even and saturates to +-448.
* per 128 x 128 tile: s = amax(tile) / 448 (1 for an all-zero tile),
  q = e4m3(a / s) with the division in float32.
"""
from __future__ import annotations

import numpy as np

# every finite e4m3 value, indexed by its code
_E4M3 = np.empty(256, dtype=np.float64)
for _c in range(256):
    _s = -1.0 if _c & 0x80 else 1.0
    _e = (_c >> 3) & 0xF
    _m = _c & 0x7
    if _e == 15 and _m == 7:
        _E4M3[_c] = np.nan
    elif _e == 0:
        _E4M3[_c] = _s * (_m / 8.0) * 2.0 ** -6
    else:
        _E4M3[_c] = _s * (1.0 + _m / 8.0) * 2.0 ** (_e - 7)


def e4m3_decode(codes: np.ndarray) -> np.ndarray:
    return _E4M3[np.asarray(codes, dtype=np.uint8)]


def e4m3_encode(x: np.ndarray) -> np.ndarray:
    """Nearest e4m3 code of each float32 value (ties to the even code,
    saturating), by search over the table of positive finite values."""
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    pos = _E4M3[:127]                       # codes 0x00..0x7E, increasing
    a = np.minimum(np.abs(x), 448.0)
    hi = np.searchsorted(pos, a, side="left")   # first value >= a
    hi = np.minimum(hi, 126)
    lo = np.maximum(hi - 1, 0)
    dlo = a - pos[lo]
    dhi = pos[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo).astype(np.uint8)
    code = np.where(a == pos[hi], hi, code).astype(np.uint8)
    code = code | (np.signbit(x).astype(np.uint8) << 7)
    code = np.where(np.isnan(x), np.uint8(0x7F), code)
    return code.astype(np.uint8)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bits (uint16), round to nearest even."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = (u & 0x7FFFFFFF) > 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(nan, 0x7FC0, r)
    return r.astype(np.uint16)


def bf16_decode(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def quantize_fp8_tiles(A: np.ndarray):
    """(codes uint8 n x d, scales float32 ceil(n/128) x ceil(d/128))."""
    A = np.asarray(A, dtype=np.float32)
    n, d = A.shape
    tn, td = -(-n // 128), -(-d // 128)
    scales = np.empty((tn, td), dtype=np.float32)
    codes = np.empty((n, d), dtype=np.uint8)
    for i in range(tn):
        for j in range(td):
            blk = A[i * 128:(i + 1) * 128, j * 128:(j + 1) * 128]
            am = np.float32(np.max(np.abs(blk))) if blk.size else np.float32(0)
            s = np.float32(am / np.float32(448.0)) if am > 0 else np.float32(1.0)
            scales[i, j] = s
            codes[i * 128:(i + 1) * 128, j * 128:(j + 1) * 128] = e4m3_encode(blk / s)
    return codes, scales


def dequantize_fp8_tiles(codes: np.ndarray, scales: np.ndarray) -> np.ndarray:
    n, d = codes.shape
    s = np.repeat(np.repeat(scales.astype(np.float64), 128, axis=0), 128, axis=1)[:n, :d]
    return e4m3_decode(codes) * s
