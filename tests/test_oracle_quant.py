"""Pins of the reduced-precision storage model: binary16 error bound, exact
round trip of representable values, zero spinors, and 12-real link reconstruction."""
import numpy as np

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
