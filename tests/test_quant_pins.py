"""Pins of the 16-bit storage oracle (oracle/quant.py), CPU only.

Rounding is checked against a brute-force nearest-value search on exact
rationals, against hand-picked tie and boundary values, and against the
error bound of each format; planted mistakes (truncation, ties away from
zero) must fail the pins.
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import quant


def _bf16_nearest_bruteforce(x: float) -> int:
    """Nearest bfloat16 to float32 x by exact comparison of its two
    neighbours on the bfloat16 grid (ties to the even word)."""
    u = int(np.float32(x).view(np.uint32))
    lo = u >> 16                      # truncation toward zero (same sign)
    hi = lo + 1                       # next bfloat16 away from zero
    fx = Fraction(float(np.float32(x)))
    flo = Fraction(float(quant.bf16_value(np.uint16(lo))))
    fhi = Fraction(float(quant.bf16_value(np.uint16(hi))))
    dlo, dhi = abs(fx - flo), abs(fx - fhi)
    if dlo < dhi:
        return lo
    if dhi < dlo:
        return hi
    return lo if lo % 2 == 0 else hi


def test_bf16_rounding_matches_bruteforce():
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.normal(0, 1, 400), rng.normal(0, 1e4, 200), rng.uniform(-3, 3, 200) * 1e-30])
    # exact ties: a float32 whose low 16 bits are 0x8000
    ties = (rng.integers(0x3F800000, 0x46800000, 100, dtype=np.int64) & ~0xFFFF) | 0x8000
    xs = np.concatenate([xs.astype(np.float32), ties.astype(np.uint32).view(np.float32)])
    got = quant.bf16_bits(xs.astype(np.float32))
    want = np.array([_bf16_nearest_bruteforce(float(x)) for x in xs], dtype=np.uint16)
    assert np.array_equal(got, want)


def test_bf16_known_values():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1.0, 2.0 ** 14, 1 + 2 ** -9], np.float32)
    assert [hex(int(b)) for b in quant.bf16_bits(v)] == ["0x3f80", "0x3f80", "0x3f82", "0xbf80", "0x4680", "0x3f80"]


def test_f16_known_values():
    v = np.array([1.0, 1 + 2 ** -11, 1 + 3 * 2 ** -11, 2.0 ** 14, 2.0 ** -24, 3 * 2.0 ** -25, -2.0], np.float32)
    assert [hex(int(b)) for b in quant.f16_bits(v)] == ["0x3c00", "0x3c00", "0x3c02", "0x7400", "0x1", "0x2", "0xc000"]


def test_scale_definition():
    f = np.zeros((3, 4, 5), np.float32)
    f[0, 1, 2] = -3.0
    f[1] = 7.25
    s = quant.frame_scales(f)
    assert s.dtype == np.float32
    assert s[0] == np.float32(3.0 * 2 ** -14) and s[1] == np.float32(7.25 * 2 ** -14) and s[2] == 1.0
    q, s2, o = quant.quantize_frames(f, "bf16")
    assert np.array_equal(s, s2) and np.all(q[2] == 0) and np.all(o == 0)
    # the largest magnitude maps to exactly 2^14
    assert quant.bf16_value(q[0, 1, 2]) == -(2.0 ** 14)


@pytest.mark.parametrize("kind,u", [("bf16", 2.0 ** -8), ("f16", 2.0 ** -11)])
def test_roundtrip_error_bound(kind, u):
    rng = np.random.default_rng(11)
    f = rng.normal(100, 10, size=(4, 64, 64)).astype(np.float32)
    f[1] *= 1e-3
    q, s, _ = quant.quantize_frames(f, kind)
    d = quant.dequantize_frames(q, s, kind)
    err = np.abs(d.astype(np.float64) - f.astype(np.float64))
    # unit roundoff of the format plus one float32 rounding of each step
    assert np.all(err <= (u + 3 * 2.0 ** -24) * np.abs(f) + 1e-30)
    assert float(err.max() / np.abs(f).max()) > u / 8  # the rounding really happens


def test_centring():
    """Centred storage: the offset is the frame mean (float32 of the float64
    mean), the stored frame is F - offset, a constant frame stores zeros with
    scale 1, and the rounding error follows |F - mean| instead of |F|."""
    rng = np.random.default_rng(12)
    f = rng.normal(100, 10, size=(3, 32, 48)).astype(np.float32)
    f[2] = 42.5
    q, s, o = quant.quantize_frames(f, "bf16", center=True)
    assert o[0] == np.float32(f[0].astype(np.float64).mean()) and o[2] == np.float32(42.5)
    assert s[2] == 1.0 and np.all(q[2] == 0)
    d = quant.dequantize_frames(q, s, "bf16").astype(np.float64)
    ref = f.astype(np.float64) - o[:, None, None]
    err_c = np.abs(d - ref)[:2]
    assert np.all(err_c <= (2.0 ** -8 + 3 * 2.0 ** -24) * np.abs(ref[:2]) + 2 * 2.0 ** -24 * np.abs(f[:2]) + 1e-30)
    qn, sn, _ = quant.quantize_frames(f, "bf16")
    err_n = np.abs(quant.dequantize_frames(qn, sn, "bf16").astype(np.float64) - f)[:2]
    assert err_c.mean() < err_n.mean() / 4


def test_planted_truncation_is_caught(monkeypatch):
    monkeypatch.setattr(quant, "bf16_bits",
                        lambda x: (np.ascontiguousarray(x, np.float32).view(np.uint32) >> 16).astype(np.uint16))
    with pytest.raises(AssertionError):
        test_bf16_known_values()


def test_planted_ties_away_is_caught(monkeypatch):
    def away(x):
        u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
        return ((u + 0x8000) >> 16).astype(np.uint16)
    monkeypatch.setattr(quant, "bf16_bits", away)
    with pytest.raises(AssertionError):
        test_bf16_known_values()
