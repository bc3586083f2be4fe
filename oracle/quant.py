"""Oracle: reference model of the reduced-precision storage formats of the mixed solver.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's run stored its fields in single precision (section 3: the 3x3
link matrix occupies 72 bytes).  The mixed solver stores spinors, links and
the clover blocks in IEEE binary16; these functions define those encodings
in NumPy so that the GPU encoders can be compared bit for bit, and evaluate
the even-odd operator on the stored values:

* spinor: s = max over the 24 real components of |c| (float32);
  inv = 1 / s in float32 (0 if s == 0); code = binary16(round-to-nearest-even(c * inv))
  with the product formed in float32.  Decoding: float32(code) * s.
* link: the first two rows (12 reals) of U, each rounded float64 -> float32 ->
  binary16; the third row is rebuilt as conj(row0 x row1), valid for det U = 1.
* clover: each chiral 6x6 Hermitian block as its 36 reals (6 diagonal, 15
  upper off-diagonal complex entries), encoded like a spinor with one scale
  per block (max |real|); the lower triangle is the conjugate of the upper.
* compact clover (A_ee of a clover term built from links): each chiral block
  is 1 - [[X3, W], [W^dag, -X3]] with X3 traceless Hermitian (3x3 blocks over
  the two spins of the half); the 26 reals [X3_00, X3_11, X3_01, X3_02, X3_12,
  W row-major] are encoded like a spinor with one scale per block.
* ``mhat_stored16``: Mhat = A_ee - kappa^2 H_eo A_oo^-1 H_oe evaluated exactly
  on those stored values -- psi, the links, A_ee, A_oo^-1, the intermediate
  t = A_oo^-1 H_oe psi and the output each taken through its format -- which
  is what the mixed stencil computes up to its float32 arithmetic.
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


def _scaled16(reals: np.ndarray) -> np.ndarray:
    """Round float reals (..., n) through the scaled binary16 encoding (one float32
    scale max |real| per leading index) and return the decoded float64 values."""
    r = reals.astype(np.float32)
    sc = np.abs(r).max(-1).astype(np.float32)
    with np.errstate(divide="ignore"):
        inv = np.where(sc > 0, np.float32(1.0) / np.where(sc > 0, sc, np.float32(1.0)), np.float32(0.0)).astype(np.float32)
    codes = (r * inv[..., None]).astype(np.float32).astype(np.float16)
    return (codes.astype(np.float32) * sc[..., None]).astype(np.float64)


def roundtrip16(psi):
    """Spinors (..., 4, 3) complex -> the values their binary16 storage decodes to."""
    codes, s = quantize16(np.asarray(psi))
    return dequantize16(codes, s)


def link_roundtrip12(u):
    """U (..., 3, 3) -> the 12-real binary16 link: stored rows decoded, row 2 rebuilt."""
    u = np.asarray(u)
    h = link_to_half12(u).astype(np.float64).reshape(u.shape[:-2] + (2, 3, 2))
    return reconstruct12(h[..., 0] + 1j * h[..., 1])


def clover_roundtrip(a12, bits: int = 16):
    """Block-diagonal clover matrices (..., 12, 12) -> their stored values: per chiral
    6x6 block binary16 with one scale (bits = 16), or every real in float32 (32)."""
    a12 = np.asarray(a12)
    out = np.zeros_like(a12)
    iu = np.triu_indices(6, 1)
    for b in range(2):
        blk = a12[..., 6 * b:6 * b + 6, 6 * b:6 * b + 6]
        d = np.diagonal(blk, axis1=-2, axis2=-1).real
        off = blk[..., iu[0], iu[1]]
        reals = np.concatenate([d, np.stack([off.real, off.imag], -1).reshape(off.shape[:-1] + (30,))], -1)
        if bits == 16:
            q = _scaled16(reals)
        else:
            q = reals.astype(np.float32).astype(np.float64)
        qoff = q[..., 6::2] + 1j * q[..., 7::2]
        nb = np.zeros(blk.shape, dtype=np.complex128)
        nb[..., np.arange(6), np.arange(6)] = q[..., :6]
        nb[..., iu[0], iu[1]] = qoff
        nb[..., iu[1], iu[0]] = np.conj(qoff)
        out[..., 6 * b:6 * b + 6, 6 * b:6 * b + 6] = nb
    return out


def compact_blocks(a12):
    """Block-diagonal clover matrices (..., 12, 12) -> (X3, W) per chiral block,
    each (..., 2, 3, 3), from B00 = 1 - X3, B11 = 1 + X3, B01 = -W."""
    a12 = np.asarray(a12)
    x3, w = [], []
    for b in range(2):
        blk = a12[..., 6 * b:6 * b + 6, 6 * b:6 * b + 6]
        x3.append(0.5 * (blk[..., 3:, 3:] - blk[..., :3, :3]))
        w.append(-blk[..., :3, 3:])
    return np.stack(x3, -3), np.stack(w, -3)


def blocks_from_compact(x3, w):
    """Inverse of compact_blocks: the 12x12 block-diagonal matrices."""
    shp = x3.shape[:-3]
    out = np.zeros(shp + (12, 12), dtype=np.complex128)
    eye = np.eye(3)
    for b in range(2):
        o = 6 * b
        out[..., o:o + 3, o:o + 3] = eye - x3[..., b, :, :]
        out[..., o + 3:o + 6, o + 3:o + 6] = eye + x3[..., b, :, :]
        out[..., o:o + 3, o + 3:o + 6] = -w[..., b, :, :]
        out[..., o + 3:o + 6, o:o + 3] = -np.conj(np.swapaxes(w[..., b, :, :], -1, -2))
    return out


def compact_roundtrip16(a12):
    """A_ee in the compact binary16 form -> the block-diagonal matrices it decodes to
    (X3's last diagonal entry rebuilt as -(X3_00 + X3_11))."""
    x3, w = compact_blocks(a12)
    reals = np.concatenate([x3[..., 0, 0].real[..., None], x3[..., 1, 1].real[..., None],
                            np.stack([x3[..., 0, 1].real, x3[..., 0, 1].imag, x3[..., 0, 2].real, x3[..., 0, 2].imag,
                                      x3[..., 1, 2].real, x3[..., 1, 2].imag], -1),
                            np.stack([w.real, w.imag], -1).reshape(w.shape[:-2] + (18,))], -1)
    q = _scaled16(reals)
    d0, d1 = q[..., 0], q[..., 1]
    x01, x02, x12 = q[..., 2] + 1j * q[..., 3], q[..., 4] + 1j * q[..., 5], q[..., 6] + 1j * q[..., 7]
    xq = np.zeros(x3.shape, dtype=np.complex128)
    xq[..., 0, 0], xq[..., 1, 1], xq[..., 2, 2] = d0, d1, -(d0 + d1)
    xq[..., 0, 1], xq[..., 0, 2], xq[..., 1, 2] = x01, x02, x12
    xq[..., 1, 0], xq[..., 2, 0], xq[..., 2, 1] = np.conj(x01), np.conj(x02), np.conj(x12)
    wq = (q[..., 8::2] + 1j * q[..., 9::2]).reshape(w.shape)
    return blocks_from_compact(xq, wq)


def mhat_stored16(setup, psi_e, dagger: bool = False, clover_bits: int = 16, compact: bool = False):
    """Mhat psi_e (Mhat^dag if dagger) evaluated exactly on the mixed solver's stored
    operands (A_ee in the compact form if compact); setup is an oracle.CloverSetup
    of the FP64 gauge field.  Returns the
    decoded output (Vh, 4, 3) complex128 and the undecoded value before the output
    is stored."""
    import torch

    from .core import from_eo, hop, to_eo

    dims = setup.dims
    u16 = torch.as_tensor(link_roundtrip12(setup.u.numpy()))
    if compact and clover_bits == 16:
        a_e = torch.as_tensor(compact_roundtrip16(setup.A_e.numpy()))
    else:
        a_e = torch.as_tensor(clover_roundtrip(setup.A_e.numpy(), clover_bits))
    ai_o = torch.as_tensor(clover_roundtrip(setup.Ainv_o.numpy(), clover_bits))
    psi = torch.as_tensor(roundtrip16(torch.as_tensor(psi_e).numpy()))

    def mv(a, v):
        return torch.einsum("...ij,...j->...i", a, v.reshape(v.shape[:-2] + (12,))).reshape(v.shape)

    h = to_eo(hop(u16, from_eo(psi, None, dims), setup.tb, dagger), dims)[1]
    t = torch.as_tensor(roundtrip16(mv(ai_o, h).numpy()))
    out = mv(a_e, psi) - setup.kappa ** 2 * to_eo(hop(u16, from_eo(None, t, dims), setup.tb, dagger), dims)[0]
    return torch.as_tensor(roundtrip16(out.numpy())), out
