"""Oracle: reference model of the reduced-precision storage formats of the mixed solver.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's run stored its fields in single precision (section 3: the 3x3
link matrix occupies 72 bytes).  The mixed solver stores spinors and links in
IEEE binary16; these functions define those encodings in NumPy so that the
GPU encoders can be compared bit for bit:

* spinor: s = max over the 24 real components of |c| (float32);
  inv = 1 / s in float32 (0 if s == 0); code = binary16(round-to-nearest-even(c * inv))
  with the product formed in float32.  Decoding: float32(code) * s.
* link: the first two rows (12 reals) of U, each rounded float64 -> float32 ->
  binary16; the third row is rebuilt as conj(row0 x row1), valid for det U = 1.
"""
from __future__ import annotations

import numpy as np


def quantize16(psi: np.ndarray):
    """psi: complex (..., 4, 3) per site -> (codes float16 (..., 24), scale float32 (...))."""
    re = np.stack([psi.real, psi.imag], -1).astype(np.float32).reshape(psi.shape[:-2] + (24,))
    s = np.abs(re).max(-1).astype(np.float32)
    with np.errstate(divide="ignore"):
        inv = np.where(s > 0, np.float32(1.0) / np.where(s > 0, s, np.float32(1.0)), np.float32(0.0)).astype(np.float32)
    codes = (re * inv[..., None]).astype(np.float32).astype(np.float16)
    return codes, s


def dequantize16(codes: np.ndarray, s: np.ndarray) -> np.ndarray:
    v = codes.astype(np.float32) * s[..., None].astype(np.float32)
    v = v.astype(np.float64).reshape(codes.shape[:-1] + (12, 2))
    return (v[..., 0] + 1j * v[..., 1]).reshape(codes.shape[:-1] + (4, 3))


def link_to_half12(u: np.ndarray) -> np.ndarray:
    """U (..., 3, 3) complex -> (..., 12) float16: rows 0 and 1, (re, im) interleaved."""
    rows = u[..., :2, :]
    re = np.stack([rows.real, rows.imag], -1).reshape(u.shape[:-2] + (12,))
    return re.astype(np.float32).astype(np.float16)


def reconstruct12(rows01: np.ndarray) -> np.ndarray:
    """Rows 0, 1 (..., 2, 3) complex -> full (..., 3, 3) with row 2 = conj(row0 x row1)."""
    a, b = rows01[..., 0, :], rows01[..., 1, :]
    c = np.conj(np.cross(a, b))
    return np.stack([a, b, c], -2)
