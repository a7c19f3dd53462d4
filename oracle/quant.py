"""Low-precision storage rules for the mixed-precision solver.

The paper only announces mixed precision as future work (Sec. 5).  The storage
formats used here are:

  * FP32: each real number rounded to IEEE binary32, round-to-nearest-even.
  * FP16 with a per-site scale: for a group of reals v_j (one site's colour
    vector, or one site's group of links), s = binary32(max_j |v_j|), and each
    code is binary16(binary32(v_j / s)) with the quotient taken in binary64 and
    both roundings to nearest even.  s = 0 gives all-zero codes.  The stored
    value is code * s.

Dequantised values are exact in binary64 (a binary16 code times a binary32
scale has at most 35 significant bits).
"""
from __future__ import annotations

import numpy as np


def to_f32(z: np.ndarray) -> np.ndarray:
    """Round complex128 to complex64 parts; return them as complex128 again."""
    return z.astype(np.complex64).astype(np.complex128)


def f16_scale(group_reals: np.ndarray, axis) -> np.ndarray:
    """Per-group binary32 scale = rounded max |v| over `axis`."""
    return np.max(np.abs(group_reals), axis=axis).astype(np.float32)


def f16_codes(group_reals: np.ndarray, scale_b: np.ndarray) -> np.ndarray:
    """binary16 codes of v / s (quotient in binary64, rounded to binary32, then to binary16)."""
    s = scale_b.astype(np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(s != 0.0, group_reals / np.where(s != 0.0, s, 1.0), 0.0)
    return q.astype(np.float32).astype(np.float16)


def quantize_spinor_f16(v: np.ndarray):
    """[..., 3] complex128 colour vectors -> (codes [..., 6] float16, scale [...] float32)."""
    reals = np.stack([v.real, v.imag], axis=-1).reshape(v.shape[:-1] + (6,))
    s = f16_scale(reals, axis=-1)
    return f16_codes(reals, s[..., None]), s


def dequantize_spinor_f16(codes: np.ndarray, s: np.ndarray) -> np.ndarray:
    vals = codes.astype(np.float64) * s.astype(np.float64)[..., None]
    vals = vals.reshape(vals.shape[:-1] + (3, 2))
    return vals[..., 0] + 1j * vals[..., 1]


def spinor_f16_roundtrip(v: np.ndarray) -> np.ndarray:
    return dequantize_spinor_f16(*quantize_spinor_f16(v))


def quantize_link_group_f16(U: np.ndarray):
    """U: [..., G, 3, 3] links that share one scale -> (codes [..., G, 3, 3, 2], scale [...])."""
    reals = np.stack([U.real, U.imag], axis=-1)
    s = f16_scale(reals.reshape(U.shape[:-3] + (-1,)), axis=-1)
    return f16_codes(reals, s[..., None, None, None, None]), s


def dequantize_link_group_f16(codes: np.ndarray, s: np.ndarray) -> np.ndarray:
    vals = codes.astype(np.float64) * s.astype(np.float64)[..., None, None, None, None]
    return vals[..., 0] + 1j * vals[..., 1]
