"""Pins for the oracle's number-format conversions (CPU only).

The RNE conversions are written from the format definitions; here they are
checked bit for bit against independent library casts (torch's bfloat16 and
float8_e4m3fn, numpy's float16), against hand-worked tie cases, and by
exhaustive round trips over every code of each format.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import formats as F


def _probe_values(seed=0, n=200_000):
    g = synth.rng(seed)
    parts = [
        synth.draw(g, (n,), "normal"),
        synth.draw(g, (n,), "wide"),
        (synth.draw(g, (n,), "normal") * np.float32(2.0 ** -130)).astype(np.float32),  # f32 subnormals
        (synth.draw(g, (n,), "normal") * np.float32(1e4)).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, 65504.0, 65520.0, 65519.0, 3e38, -3e38], np.float32),
    ]
    # every float32 bit pattern with a random upper part and all low 16-bit tie cases
    hi = g.integers(0x0080, 0x7F00, size=2000, dtype=np.uint32) << 16
    lo = np.array([0x0000, 0x7FFF, 0x8000, 0x8001, 0xFFFF], dtype=np.uint32)
    parts.append((hi[:, None] | lo[None, :]).ravel().view(np.float32))
    return np.concatenate(parts).astype(np.float32)


def test_bf16_matches_torch_cast():
    x = _probe_values(1)
    ours = F.to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_f16_matches_numpy_cast():
    x = _probe_values(2)
    ours = F.to_f16_bits(x)
    ref = x.astype(np.float16).view(np.uint16)
    assert np.array_equal(ours, ref)


def test_e4m3_matches_torch_cast_in_range():
    x = _probe_values(3)
    x = x[np.abs(x) <= 448.0]
    ours = F.encode(F.round_to_format(x.astype(np.float64), "e4m3"), "e4m3")
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, ref)


def test_tie_cases_by_hand():
    # bfloat16: ulp(1) = 2^-7
    assert F.round_to_format(1 + 2.0 ** -8, "bf16") == 1.0               # tie -> even (down)
    assert F.round_to_format(1 + 3 * 2.0 ** -8, "bf16") == 1 + 2.0 ** -6  # tie -> even (up)
    assert F.round_to_format(1 + 2.0 ** -8 + 2.0 ** -20, "bf16") == 1 + 2.0 ** -7
    # E4M3: smallest subnormal 2^-9
    assert F.round_to_format(2.0 ** -10, "e4m3") == 0.0
    assert F.round_to_format(3 * 2.0 ** -10, "e4m3") == 2.0 ** -8
    assert F.round_to_format(1.0625, "e4m3") == 1.0     # 1 + 2^-4 is the midpoint of 1 and 1.125
    # saturation to +-448 and IEEE overflow
    assert F.round_to_format(500.0, "e4m3") == 448.0
    assert F.round_to_format(-1e6, "e4m3") == -448.0
    assert F.round_to_format(464.0, "e4m3") == 448.0
    assert F.round_to_format(65520.0, "f16") == np.inf
    assert F.round_to_format(65519.0, "f16") == 65504.0


@pytest.mark.parametrize("fmt,width", [("e4m3", 8), ("bf16", 16), ("f16", 16)])
def test_exhaustive_round_trip(fmt, width):
    codes = np.arange(1 << width, dtype=np.uint32).astype({8: np.uint8, 16: np.uint16}[width])
    vals = F.decode(codes, fmt)
    if fmt == "e4m3":
        keep = (codes & 0x7F) != 0x7F                       # drop the two NaN codes
    else:
        ebits = 8 if fmt == "bf16" else 5
        mb = 15 - ebits
        keep = ((codes.astype(np.uint32) >> mb) & ((1 << ebits) - 1)) != (1 << ebits) - 1
    codes, vals = codes[keep], vals[keep]
    assert np.array_equal(F.round_to_format(vals, fmt), vals)   # already representable
    assert np.array_equal(F.encode(vals, fmt), codes)
    # the decoded values are strictly increasing over the positive codes
    pos = vals[(codes.astype(np.uint32) >> (width - 1)) == 0]
    assert np.all(np.diff(pos) > 0)


def test_e4m3_decode_known_codes():
    assert F.decode(np.array([0x7E]), "e4m3")[0] == 448.0
    assert F.decode(np.array([0x01]), "e4m3")[0] == 2.0 ** -9
    assert F.decode(np.array([0x08]), "e4m3")[0] == 2.0 ** -6
    assert F.decode(np.array([0x38]), "e4m3")[0] == 1.0
    assert F.decode(np.array([0xB8]), "e4m3")[0] == -1.0


def test_e4m3_scale_and_quantise():
    x = np.array([0.0, 1.0, -3.5, 2.0], np.float32)
    s = F.e4m3_scale(x)
    assert s == np.float32(np.float32(3.5) / np.float32(448.0))
    q = F.decode(F.to_e4m3_bits(x, s), "e4m3")
    assert q[2] == -448.0 and q[0] == 0.0
    assert F.e4m3_scale(np.zeros(4, np.float32)) == 1.0
    # every quantised magnitude stays within the finite range
    g = synth.rng(5)
    y = synth.draw(g, (10000,), "wide")
    qs = F.decode(F.to_e4m3_bits(y, F.e4m3_scale(y)), "e4m3")
    assert np.max(np.abs(qs)) == 448.0


def test_split_bf16_identity_and_bound():
    x = _probe_values(4)
    x = x[np.isfinite(x) & (np.abs(x) < 1e38) & (np.abs(x) > 1e-30)]
    hi, lo = F.split_bf16(x)
    h = F.decode(hi, "bf16")
    l_ = F.decode(lo, "bf16")
    res = x.astype(np.float64) - h - l_
    assert np.all(np.abs(res) <= 2.0 ** -16 * np.abs(x.astype(np.float64)))
    # x - hi is exact in binary32, so lo is the RNE of an exactly known value
    d32 = (x - h.astype(np.float32)).astype(np.float64)
    assert np.array_equal(d32, x.astype(np.float64) - h)
