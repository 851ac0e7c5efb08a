"""Number formats of the precision forms, written from their definitions.

TEST INFRASTRUCTURE ONLY (part of the oracle): only the test suite, the smoke
check and the CPU-baseline leg of the benchmark import this module.

The paper computes in float, double and complex float only (Results section,
Table 2).  The reduced-precision forms of the product are this project's
extension; their formats are the public ones:

* bfloat16: 1 sign, 8 exponent, 7 fraction bits (p = 8 significant bits,
  e_min = -126), IEEE-style inf/NaN.
* binary16: 1 sign, 5 exponent, 10 fraction bits (p = 11, e_min = -14).
* OCP FP8 E4M3 ("e4m3fn"): 1 sign, 4 exponent (bias 7), 3 fraction bits
  (p = 4, e_min = -6); no infinities; the all-ones exponent with fraction
  111 is NaN, so the largest finite magnitude is 1.75 * 2^8 = 448.

Rounding is round-to-nearest, ties-to-even (RNE), done here by scaling the
binary64 value so that the last kept bit is the units digit, rounding with
numpy's ``rint`` (which rounds halves to even) and scaling back; all steps are
exact in binary64 for every float32 input.  Overflow goes to +-inf for the two
IEEE-style formats and saturates to +-448 for E4M3 (OCP "satfinite").

The per-tensor FP8 scale is s = amax / 448 computed in binary32 (amax = max
|x|; an all-zero tensor gets s = 1), and the code of x is E4M3(RNE_sat(x / s))
with the quotient rounded to binary32 first: both sides of a comparison take
the quantisation decision in binary32, the arithmetic of the GPU kernels.

The compensated form ("split-BF16x3") writes x = hi + lo + residual with
hi = RNE_bf16(x) and lo = RNE_bf16(x - hi); x - hi is exact in binary32.
"""
from __future__ import annotations

import numpy as np

# name -> (p significant bits, e_min, exponent bits, bias, max finite, saturating)
_FMT = {
    "bf16": (8, -126, 8, 127, float((2 - 2.0 ** -7) * 2.0 ** 127), False),
    "f16": (11, -14, 5, 15, 65504.0, False),
    "e4m3": (4, -6, 4, 7, 448.0, True),
}

E4M3_MAX = 448.0


def round_to_format(x, fmt: str) -> np.ndarray:
    """Round binary64 values to the nearest value of ``fmt`` (RNE).

    Returns the rounded values as binary64 (exact).
    """
    p, emin, _ebits, _bias, vmax, sat = _FMT[fmt]
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)              # x = f * 2**e, 0.5 <= |f| < 1
    lead = np.maximum(e - 1, emin)  # exponent of the leading bit (clamped: subnormals)
    q = np.ldexp(x, (p - 1) - lead)  # last kept bit now has weight 1
    y = np.ldexp(np.rint(q), lead - (p - 1))
    big = np.abs(y) > vmax
    if sat:
        y = np.where(big, np.copysign(vmax, x), y)
    else:
        y = np.where(big, np.copysign(np.inf, x), y)
    return y


def encode(y, fmt: str) -> np.ndarray:
    """Bit patterns of values already representable in ``fmt``."""
    p, emin, ebits, bias, _vmax, _sat = _FMT[fmt]
    mbits = p - 1
    y = np.asarray(y, dtype=np.float64)
    sign = np.signbit(y).astype(np.uint32)
    a = np.abs(y)
    out = np.zeros(a.shape, dtype=np.uint32)
    inf = np.isinf(a)
    _, e = np.frexp(a)
    lead = e - 1
    normal = (a > 0) & (lead >= emin) & ~inf
    sub = (a > 0) & (lead < emin)
    expf = np.where(normal, lead + bias, 0).astype(np.int64)
    frac_normal = np.ldexp(a, mbits - lead) - (1 << mbits)      # (a/2^lead - 1) * 2^mbits
    frac_sub = np.ldexp(a, mbits - emin)                        # a / 2^(emin - mbits)
    frac = np.where(normal, frac_normal, np.where(sub, frac_sub, 0.0))
    out = (expf.astype(np.uint32) << mbits) | frac.astype(np.uint32)
    out = np.where(inf, np.uint32(((1 << ebits) - 1) << mbits), out)
    out = out | (sign << (ebits + mbits))
    width = {8: np.uint8, 16: np.uint16}[1 + ebits + mbits]
    return out.astype(width)


def decode(bits, fmt: str) -> np.ndarray:
    """Values (binary64) of finite bit patterns of ``fmt``."""
    p, emin, ebits, bias, _vmax, _sat = _FMT[fmt]
    mbits = p - 1
    b = np.asarray(bits).astype(np.int64)
    sign = (b >> (ebits + mbits)) & 1
    expf = (b >> mbits) & ((1 << ebits) - 1)
    frac = b & ((1 << mbits) - 1)
    normal = np.ldexp(1.0 + frac / float(1 << mbits), (expf - bias).astype(np.int64))
    sub = np.ldexp(frac.astype(np.float64), emin - mbits)
    v = np.where(expf == 0, sub, normal)
    if fmt != "e4m3":
        v = np.where(expf == (1 << ebits) - 1, np.inf, v)
    return np.where(sign == 1, -v, v)


def to_bf16_bits(x_f32) -> np.ndarray:
    """float32 -> bfloat16 codes, RNE."""
    return encode(round_to_format(np.asarray(x_f32, np.float32).astype(np.float64), "bf16"), "bf16")


def to_f16_bits(x_f32) -> np.ndarray:
    """float32 -> binary16 codes, RNE."""
    return encode(round_to_format(np.asarray(x_f32, np.float32).astype(np.float64), "f16"), "f16")


def e4m3_scale(x_f32) -> np.float32:
    """Per-tensor scale s = amax / 448 in binary32; 1 for an all-zero tensor."""
    amax = np.float32(np.max(np.abs(np.asarray(x_f32, np.float32)))) if np.size(x_f32) else np.float32(0)
    if amax == 0:
        return np.float32(1.0)
    return np.float32(amax / np.float32(E4M3_MAX))


def to_e4m3_bits(x_f32, scale) -> np.ndarray:
    """E4M3 codes of x / scale, the quotient rounded to binary32 first."""
    q = (np.asarray(x_f32, np.float32) / np.float32(scale)).astype(np.float32)
    return encode(round_to_format(q.astype(np.float64), "e4m3"), "e4m3")


def split_bf16(x_f32):
    """(hi, lo) bfloat16 codes with hi = RNE(x), lo = RNE(x - hi)."""
    x = np.asarray(x_f32, np.float32).astype(np.float64)
    hi = round_to_format(x, "bf16")
    lo = round_to_format(x - hi, "bf16")
    return encode(hi, "bf16"), encode(lo, "bf16")
