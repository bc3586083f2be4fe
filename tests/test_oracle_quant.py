"""Pins of the reduced-precision storage model: binary16 error bound, exact
round trip of representable values, zero spinors, 12-real link reconstruction,
the clover blocks' storage, and the even-odd operator on stored operands
(equal to the FP64 operator when nothing is rounded, and inside the a-priori
rounding bound when everything is)."""
import numpy as np
import pytest
import torch

import oracle as O
import oracle.quant as Q
from oracle.quant import dequantize16, link_to_half12, quantize16, reconstruct12
from paper_0910_0262_amd import synth


def test_quantizer_error_bound():
    rng = np.random.default_rng(0)
    psi = rng.standard_normal((1000, 4, 3)) * np.exp(rng.uniform(-20, 20, (1000, 1, 1))) \
        + 1j * rng.standard_normal((1000, 4, 3))
    codes, s = quantize16(psi)
    back = dequantize16(codes, s)
    err = np.abs(np.stack([(back - psi).real, (back - psi).imag], -1)).reshape(1000, 24).max(-1)
    assert np.all(err <= s * 2.0 ** -11 * (1 + 2.0 ** -9))
    assert np.all(np.abs(codes.astype(np.float32)).max(-1) == 1.0)


def test_quantizer_exact_on_representable_values():
    v = np.array([1.0, -0.5, 0.25, 0.125, 0.75, -1.0] * 4)
    psi = (v[0::2] + 1j * v[1::2]).reshape(1, 4, 3) * 8.0
    codes, s = quantize16(psi)
    assert s[0] == 8.0
    assert np.array_equal(dequantize16(codes, s), psi)


def test_quantizer_zero_spinor():
    codes, s = quantize16(np.zeros((3, 4, 3), complex))
    assert np.all(s == 0) and np.all(codes == 0)
    assert np.all(dequantize16(codes, s) == 0)


def test_link_reconstruction():
    u = synth.random_su3_field((2, 2, 2, 2), 0.7, 3).reshape(-1, 3, 3)
    full = reconstruct12(u[:, :2, :])
    assert np.abs(full - u).max() < 1e-14
    h = link_to_half12(u).astype(np.float64).reshape(-1, 2, 3, 2)
    rows = h[..., 0] + 1j * h[..., 1]
    approx = reconstruct12(rows)
    assert np.abs(approx - u).max() < 4e-3


# ---------------------------------------------------------------- clover storage and the stored-operand operator
def _herm_blocks(n, seed):
    rng = np.random.default_rng(seed)
    a = np.zeros((n, 12, 12), complex)
    for b in range(2):
        m = rng.standard_normal((n, 6, 6)) + 1j * rng.standard_normal((n, 6, 6))
        a[:, 6 * b:6 * b + 6, 6 * b:6 * b + 6] = (m + np.conj(np.swapaxes(m, -1, -2))) * np.exp(rng.uniform(-6, 6, (n, 1, 1)))
    return a


def test_clover_roundtrip_bound_and_structure():
    a = _herm_blocks(200, 1)
    for bits, u in ((16, 2.0 ** -11), (32, 2.0 ** -24)):
        q = Q.clover_roundtrip(a, bits)
        assert np.array_equal(q, np.conj(np.swapaxes(q, -1, -2)))  # Hermitian
        assert np.all(q[:, :6, 6:] == 0) and np.all(q[:, 6:, :6] == 0)  # chiral blocks only
        for b in range(2):
            blk, qb = a[:, 6 * b:6 * b + 6, 6 * b:6 * b + 6], q[:, 6 * b:6 * b + 6, 6 * b:6 * b + 6]
            scale = np.maximum(np.abs(blk.real), np.abs(blk.imag)).max((-2, -1))
            err = np.maximum(np.abs((qb - blk).real), np.abs((qb - blk).imag)).max((-2, -1))
            if bits == 16:
                assert np.all(err <= scale * u * (1 + 2.0 ** -9))
                # one entry of each block decodes to +-scale exactly
                assert np.all(np.maximum(np.abs(qb.real), np.abs(qb.imag)).max((-2, -1)) == scale.astype(np.float32))
            else:
                assert np.all(err <= np.maximum(np.abs(blk.real), np.abs(blk.imag)).max((-2, -1)) * u)
    eye = np.broadcast_to(np.eye(12, dtype=complex), (3, 12, 12))
    assert np.array_equal(Q.clover_roundtrip(eye, 16), eye)


def test_link_roundtrip_unit_and_bound():
    eye = np.broadcast_to(np.eye(3, dtype=complex), (4, 3, 3))
    assert np.array_equal(Q.link_roundtrip12(eye), eye)
    u = synth.random_su3_field((2, 2, 2, 2), 0.7, 4)
    assert np.abs(Q.link_roundtrip12(u) - u).max() < 4e-3


def test_mhat_stored16_structure_without_rounding(monkeypatch):
    """With every storage format made exact the stored-operand operator is the
    oracle's Mhat / Mhat^dag: the operand order, signs and adjoint are right."""
    dims = (4, 4, 2, 4)
    s = O.CloverSetup(torch.as_tensor(synth.random_su3_field(dims, 0.4, 5)), 0.13, 1.2)
    psi = torch.as_tensor(np.random.default_rng(6).standard_normal((s.Vh, 4, 3, 2)) @ [1, 1j])
    monkeypatch.setattr(Q, "roundtrip16", lambda p: np.asarray(p))
    monkeypatch.setattr(Q, "link_roundtrip12", lambda u: np.asarray(u))
    monkeypatch.setattr(Q, "clover_roundtrip", lambda a, bits=16: np.asarray(a))
    for dag, ref in ((False, s.Mhat(psi)), (True, s.Mhat_dag(psi))):
        got, pre = Q.mhat_stored16(s, psi, dag)
        assert float(torch.abs(got - ref).max()) < 1e-13 * float(torch.abs(ref).max())


@pytest.mark.parametrize("bits", [16, 32])
def test_mhat_stored16_within_the_rounding_bound(bits):
    """Its deviation from the FP64 Mhat stays inside the a-priori bound derived from
    the binary16 storage errors (tests/_gpu_helpers.mixed_mhat_bound), and is of the
    size binary16 storage implies (far from zero, far below the operator's values)."""
    from ._gpu_helpers import mixed_mhat_bound

    dims = (4, 4, 4, 4)
    s = O.CloverSetup(torch.as_tensor(synth.random_su3_field(dims, 0.3, 0)), 0.12, 1.0)
    psi = torch.as_tensor(np.random.default_rng(7).standard_normal((s.Vh, 4, 3, 2)) @ [1, 1j])
    for dag in (False, True):
        got, _ = Q.mhat_stored16(s, psi, dag, bits)
        bound, _, ref = mixed_mhat_bound(s, psi, dag, bits)
        err = torch.abs(got - ref).amax((-2, -1))
        assert bool((err <= bound).all())
        rel = float((err / torch.abs(ref).amax((-2, -1))).median())
        assert 2.0 ** -16 < rel < 2.0 ** -9


def test_compact_clover_form_of_built_clover():
    """A clover term built from links has, per chiral block, B00 + B11 = 2, B10 = B01^dag
    and tr(B11 - B00) = 0 (sigma_mu,nu is traceless on each chiral half and F is
    traceless), so the compact form (X3, W) holds it exactly; a general Hermitian
    block does not have the form."""
    for dims, w, kappa, csw, seed in [((4, 4, 4, 4), 0.5, 0.124, 1.3, 3), ((2, 4, 2, 2), 1.0, 0.13, 2.0, 4)]:
        u = torch.as_tensor(synth.random_su3_field(dims, w, seed))
        a = O.clover_matrix(u, kappa, csw).reshape(-1, 12, 12).numpy()
        x3, wm = Q.compact_blocks(a)
        assert np.abs(np.trace(x3, axis1=-2, axis2=-1)).max() < 1e-15
        assert np.abs(x3 - np.conj(np.swapaxes(x3, -1, -2))).max() == 0.0
        assert np.abs(Q.blocks_from_compact(x3, wm) - a).max() < 1e-15
        q = Q.compact_roundtrip16(a)
        assert np.array_equal(q, np.conj(np.swapaxes(q, -1, -2)))
        # binary16 error relative to the entries X3, W (not to the unit diagonal)
        scale = max(np.abs(x3).max(), np.abs(wm).max())
        assert 0 < np.abs(q - a).max() < 2 * scale * 2.0 ** -11
    g = _herm_blocks(4, 9)
    x3, wm = Q.compact_blocks(g)
    assert np.abs(Q.blocks_from_compact(x3, wm) - g).max() > 1e-3
