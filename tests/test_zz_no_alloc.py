"""The allocation-free gauge force (qcd_gauge_force_noalloc) against the
allocating entry point it varies, qcd_gauge_action_force, through the C ABI.

The two launch the same kernels and differ only in where the force
accumulator lives (a fixed device array of the library instead of a buffer
the context allocates), so G and F must be bit-identical.  Checked on two
calls in a row, the second on a smaller lattice than the first (the shared
array keeps the first call's contents), and on a lattice beyond the array,
which must be rejected before any device work."""
import pytest
import torch

from paper_0910_0262_amd import Lattice, QCDError, capi, synth

from ._gpu_helpers import to_dev

pytestmark = pytest.mark.gpu

BETA = 5.6


def _nan_buffers(v):
    g = torch.full((v, 4, 3, 3), complex(float("nan"), float("nan")), dtype=torch.complex128, device="cuda")
    f = torch.full((v, 4, 8), float("nan"), dtype=torch.float64, device="cuda")
    return g, f


def _same(a, b):
    return torch.equal(a.reshape(-1), b.reshape(-1))


def _noalloc(lat, want_g=True, want_f=True):
    g, f = _nan_buffers(lat.V)
    capi.qcd_gauge_force_noalloc(lat.ctx, BETA, g if want_g else None, f if want_f else None, lat.V)
    torch.cuda.synchronize()
    return g, f


def test_noalloc_gauge_force_matches_allocating_entry_point():
    # the first lattice fills most of the array, the second reuses its start
    for dims, width, seed in [((16, 16, 16, 16), 0.3, 2), ((6, 2, 2, 6), 0.5, 1)]:
        print(f"[noalloc gauge force dims={dims}]", flush=True)
        lat = Lattice(dims, 0.125, 1.0)
        lat.load_gauge(to_dev(synth.random_su3_field(dims, width, seed)), build_clover=False)
        g_n, f_n = _noalloc(lat)
        _, g_a, f_a = lat.gauge_action_force(BETA)
        torch.cuda.synchronize()
        assert _same(g_n, g_a) and _same(f_n, f_a)
        assert bool(torch.isfinite(f_n).all())
        # again, with G only and with F only
        g2, f2 = _noalloc(lat, want_f=False)
        assert _same(g2, g_a) and bool(torch.isnan(f2).all())
        g3, f3 = _noalloc(lat, want_g=False)
        assert _same(f3, f_a) and bool(torch.isnan(g3.real).all())
        lat.close()


def test_noalloc_gauge_force_rejects_what_it_cannot_hold():
    dims = (16, 16, 16, 32)  # 131072 sites: beyond the 116480 the fixed array holds
    lat = Lattice(dims, 0.125, 1.0)
    lat.load_gauge(to_dev(synth.unit_gauge(dims)), build_clover=False)
    g, f = _nan_buffers(lat.V)
    with pytest.raises(QCDError, match="EINVAL.*too large"):
        capi.qcd_gauge_force_noalloc(lat.ctx, BETA, g, f, lat.V)
    torch.cuda.synchronize()
    assert bool(torch.isnan(f).all())
    with pytest.raises(QCDError, match="EINVAL"):
        capi.qcd_gauge_force_noalloc(lat.ctx, BETA, None, None, lat.V)
    lat.close()
    small = Lattice((4, 4, 4, 4), 0.125, 1.0)
    g, f = _nan_buffers(small.V)
    with pytest.raises(QCDError, match="ESTATE"):
        capi.qcd_gauge_force_noalloc(small.ctx, BETA, g, f, small.V)
    small.close()
