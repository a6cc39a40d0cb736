"""Pins of the low-precision reference (format definitions: bfloat16 = top
half of binary32 with round-to-nearest-even; OCP e4m3 with bias 7, no
infinities, max 448)."""
import numpy as np

from oracle import quant


def test_e4m3_table_landmarks():
    t = quant.e4m3_decode(np.arange(256, dtype=np.uint8))
    assert t[0x7E] == 448.0                  # largest finite
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF])
    assert t[0x08] == 2.0 ** -6              # smallest normal
    assert t[0x01] == 2.0 ** -9              # smallest subnormal
    assert t[0x38] == 1.0                    # exponent field 7 = bias
    assert t[0xB8] == -1.0
    assert np.all(np.diff(t[:127]) > 0)      # codes 0..126 increase


def test_e4m3_round_trip_and_rounding():
    codes = np.arange(256, dtype=np.uint8)
    vals = quant.e4m3_decode(codes)
    ok = ~np.isnan(vals) & (codes != 0x80)   # -0 encodes as 0x80 too; skip it
    assert np.array_equal(quant.e4m3_encode(vals[ok].astype(np.float32)), codes[ok])
    # ties go to the even mantissa: 1 + 1/16 lies between 1 and 1.125
    assert quant.e4m3_encode(np.float32(1.0625)) == 0x38
    assert quant.e4m3_encode(np.float32(1.1875)) == 0x3A    # 1.125 | 1.25 -> 1.25
    # saturation and NaN
    assert quant.e4m3_encode(np.float32(1e6)) == 0x7E
    assert quant.e4m3_encode(np.float32(-500.0)) == 0xFE
    assert quant.e4m3_encode(np.float32(np.nan)) == 0x7F
    # below half the smallest subnormal -> 0
    assert quant.e4m3_encode(np.float32(2.0 ** -11)) == 0x00


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e38], dtype=np.float32)
    b = quant.bf16_round(x)
    assert list(b[:4]) == [0x3F80, 0x3F80, 0x3F82, 0xC020]   # tie to even twice
    back = quant.bf16_decode(b)
    assert np.all(np.abs(back - x) <= np.abs(x) * 2.0 ** -8)


def test_fp8_tiles_error_bound():
    rng = np.random.default_rng(0)
    A = (rng.standard_normal((300, 260)) * np.exp(rng.standard_normal((300, 1)))).astype(np.float32)
    codes, scales = quant.quantize_fp8_tiles(A)
    assert scales.shape == (3, 3)
    back = quant.dequantize_fp8_tiles(codes, scales)
    # per tile: |error| <= half an e4m3 ulp at the element's magnitude, which
    # is <= 2^-4 |a| for normals and 2^-10 s for subnormals
    s = np.repeat(np.repeat(scales.astype(np.float64), 128, 0), 128, 1)[:300, :260]
    assert np.all(np.abs(back - A) <= np.maximum(np.abs(A) * 2.0 ** -4, s * 2.0 ** -10) + 1e-30)
    assert np.isclose(np.max(np.abs(back[:128, :128])), np.max(np.abs(A[:128, :128])))
