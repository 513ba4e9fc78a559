"""16-bit frame storage with a per-frame scale (test infrastructure only).

TEST INFRASTRUCTURE ONLY: imported by tests and the benchmark's precision
report, never by the GPU library.

This is a data-layout step before the search, not part of the paper's method
(the paper stores its frames as calibrated images, Sec. 2.1).  Definitions:

  o_i      = float32 of the frame's float64 mean when centring, else 0
  scale_i  = max_p |F_i(p) - o_i| * 2^-14, or 1 for a constant frame
  q_i(p)   = round-to-nearest-even of the float32 quotient
             fl32(F_i(p) - o_i) / scale_i
             in bfloat16 (8 significant bits) or IEEE half (11 bits)
  F'_i(p)  = float32 product scale_i * q_i(p)    (the frame the search sees)

bfloat16 is the upper half of a float32 bit pattern; rounding to nearest
with ties to even adds 0x7FFF plus the lowest kept bit before truncating
(finite inputs).  IEEE half uses NumPy's conversion, which rounds to nearest
even.
"""

from __future__ import annotations

import numpy as np

TWO_M14 = np.float32(2.0 ** -14)


def frame_offsets(frames: np.ndarray, center: bool) -> np.ndarray:
    """float32 [n]: the float64 frame means rounded to float32, or zeros."""
    n = frames.shape[0]
    if not center:
        return np.zeros(n, np.float32)
    return frames.reshape(n, -1).astype(np.float64).mean(axis=1).astype(np.float32)


def frame_scales(frames: np.ndarray, offsets=None) -> np.ndarray:
    """float32 [n]: max |F_i - o_i| * 2^-14 (exact: a power-of-two multiple)."""
    f = frames if offsets is None else (frames - np.asarray(offsets, np.float32)[:, None, None]).astype(np.float32)
    m = np.abs(f.reshape(f.shape[0], -1)).max(axis=1).astype(np.float32)
    return np.where(m > 0, m * TWO_M14, np.float32(1.0)).astype(np.float32)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16, nearest even; raw uint16 words."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, np.uint16).astype(np.uint32) << 16).view(np.float32)


def f16_bits(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, np.float32).astype(np.float16).view(np.uint16)


def f16_value(bits: np.ndarray) -> np.ndarray:
    return np.asarray(bits, np.uint16).view(np.float16).astype(np.float32)


def quantize_frames(frames: np.ndarray, kind: str, center: bool = False):
    """(q, scale, offset): q uint16 words [n][h][w], scale and offset float32
    [n]; kind 'bf16' or 'f16'."""
    f = np.asarray(frames, np.float32)
    o = frame_offsets(f, center)
    d = (f - o[:, None, None]).astype(np.float32)  # float32 difference
    s = frame_scales(d)
    ratio = (d / s[:, None, None]).astype(np.float32)  # correctly rounded float32 quotient
    q = bf16_bits(ratio) if kind == "bf16" else f16_bits(ratio)
    return q, s, o


def dequantize_frames(q: np.ndarray, scale: np.ndarray, kind: str) -> np.ndarray:
    """float32 frames F' = scale_i * value(q) (one float32 product)."""
    v = bf16_value(q) if kind == "bf16" else f16_value(q)
    return (np.asarray(scale, np.float32)[:, None, None] * v).astype(np.float32)
