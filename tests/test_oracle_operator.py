"""Pins of the oracle's Wilson-clover operator against closed forms and symmetries.

* free field (U = 1): the momentum-space eigenvalues of M and of the even-odd
  Schur complement Mhat, from the closed form
      M(p) = 1 - 2 kappa sum cos p_mu + 2 i kappa sum gamma_mu sin p_mu,
  p_{x,y,z} = 2 pi n / L, p_t = (2n+1) pi / Lt (antiperiodic time);
* plane waves on even sites at any volume: Mhat e^{ipx} u = e^{ipx}(1 - kappa^2 D(p)^2) u,
  D(p) = 2 sum cos p_mu - 2 i sum gamma_mu sin p_mu; and the same for a pure-gauge field;
* gamma_5-hermiticity, gauge covariance under random SU(3) transforms, the
  dense adjoint of Mhat."""
import itertools

import numpy as np
import pytest
import torch

import oracle as O
from oracle.solve import dense_full_operator, dense_matrix
from paper_0910_0262_amd import synth

C = torch.complex128


def _momenta(dims, t_boundary=-1):
    lx, ly, lz, lt = dims
    px = [2 * np.pi * n / lx for n in range(lx)]
    py = [2 * np.pi * n / ly for n in range(ly)]
    pz = [2 * np.pi * n / lz for n in range(lz)]
    off = 1 if t_boundary == -1 else 0
    pt = [(2 * n + off) * np.pi / lt for n in range(lt)]
    return itertools.product(px, py, pz, pt)


def _free_eigs_M(dims, kappa, t_boundary=-1):
    out = []
    for p in _momenta(dims, t_boundary):
        c = 2 * sum(np.cos(q) for q in p)
        s = 2 * np.sqrt(sum(np.sin(q) ** 2 for q in p))
        out += [1 - kappa * (c - 1j * s)] * 6 + [1 - kappa * (c + 1j * s)] * 6
    return np.array(out)


def _free_eigs_Mhat(dims, kappa):
    out = []
    for p in _momenta(dims):
        c = 2 * sum(np.cos(q) for q in p)
        s = 2 * np.sqrt(sum(np.sin(q) ** 2 for q in p))
        out += [1 - kappa ** 2 * (c - 1j * s) ** 2] * 3 + [1 - kappa ** 2 * (c + 1j * s) ** 2] * 3
    return np.array(out)


def _match_multisets(a, b, tol):
    """Greedy nearest matching of two eigenvalue multisets."""
    a = list(np.asarray(a))
    b = np.asarray(b).copy()
    used = np.zeros(len(b), bool)
    worst = 0.0
    for z in a:
        d = np.abs(b - z)
        d[used] = np.inf
        j = int(np.argmin(d))
        used[j] = True
        worst = max(worst, d[j])
    assert worst < tol, worst


@pytest.mark.parametrize("t_boundary", [-1, 1])
def test_free_field_spectrum_M_2x4(t_boundary):
    dims = (2, 2, 2, 2)
    s = O.CloverSetup(torch.as_tensor(synth.unit_gauge(dims)), 0.12, 1.0, t_boundary)
    ev = torch.linalg.eigvals(dense_full_operator(s)).numpy()
    _match_multisets(ev, _free_eigs_M(dims, 0.12, t_boundary), 1e-12)


def test_free_field_spectrum_M_4x2x2x4():
    dims = (4, 2, 2, 4)
    s = O.CloverSetup(torch.as_tensor(synth.unit_gauge(dims)), 0.13, 1.0)
    ev = torch.linalg.eigvals(dense_full_operator(s)).numpy()
    _match_multisets(ev, _free_eigs_M(dims, 0.13), 1e-11)


@pytest.mark.slow
def test_free_field_spectrum_Mhat_4x4():
    dims = (4, 4, 4, 4)
    s = O.CloverSetup(torch.as_tensor(synth.unit_gauge(dims)), 0.12, 1.0)
    mh = dense_matrix(s.Mhat, s.Vh)
    ev = torch.linalg.eigvals(mh).numpy()
    # momenta p and p + (pi,pi,pi,pi) give the same even-site plane wave; listing all V
    # momenta with multiplicity 3 per sign covers the 12 Vh eigenvalues exactly once
    ref = _free_eigs_Mhat(dims, 0.12)
    assert len(ref) == len(ev)
    _match_multisets(ev, ref, 1e-11)


def _plane_wave_check(dims, kappa, u, omega=None, seed=0):
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    n = [rng.integers(0, L) for L in dims]
    p = [2 * np.pi * n[0] / lx, 2 * np.pi * n[1] / ly, 2 * np.pi * n[2] / lz, (2 * n[3] + 1) * np.pi / lt]
    spin_col = torch.as_tensor(rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3)))
    f64 = torch.float64
    t = torch.arange(lt, dtype=f64).view(lt, 1, 1, 1)
    z = torch.arange(lz, dtype=f64).view(1, lz, 1, 1)
    y = torch.arange(ly, dtype=f64).view(1, 1, ly, 1)
    x = torch.arange(lx, dtype=f64).view(1, 1, 1, lx)
    phase = torch.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    psi = phase[..., None, None] * spin_col
    g = O.gammas()
    d = sum(2 * np.cos(p[m]) * torch.eye(4, dtype=C) - 2j * np.sin(p[m]) * g[m] for m in range(4))
    expect = phase[..., None, None] * torch.einsum("st,tc->sc", torch.eye(4, dtype=C) - kappa ** 2 * d @ d, spin_col)
    if omega is not None:
        om = torch.as_tensor(omega)
        psi = torch.einsum("...ab,...sb->...sa", om, psi)
        expect = torch.einsum("...ab,...sb->...sa", om, expect)
    s = O.CloverSetup(torch.as_tensor(u), kappa, 1.0)
    e, _ = O.to_eo(psi, dims)
    got = s.Mhat(e)
    ref, _ = O.to_eo(expect, dims)
    assert torch.abs(got - ref).max() < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 2, 6), (2, 2, 2, 2)])
def test_plane_wave_free(dims):
    _plane_wave_check(dims, 0.125, synth.unit_gauge(dims))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 2, 4, 4)])
def test_plane_wave_pure_gauge(dims):
    om = synth.random_su3_sites(dims, 7)
    u = synth.gauge_transform(synth.unit_gauge(dims), om)
    _plane_wave_check(dims, 0.11, u, omega=om, seed=3)


@pytest.mark.parametrize("dims,width,kappa", [((4, 4, 4, 4), 0.3, 0.12), ((2, 4, 2, 4), 0.5, 0.124)])
def test_gamma5_hermiticity(dims, width, kappa):
    u = torch.as_tensor(synth.random_su3_field(dims, width, 1))
    s = O.CloverSetup(u, kappa, 1.0)
    g5 = O.gamma5()
    rng = np.random.default_rng(4)
    lx, ly, lz, lt = dims
    shp = (lt, lz, ly, lx, 4, 3)
    chi = torch.as_tensor(rng.standard_normal(shp) + 1j * rng.standard_normal(shp))
    psi = torch.as_tensor(rng.standard_normal(shp) + 1j * rng.standard_normal(shp))

    def g5m(v):
        return torch.einsum("st,...tc->...sc", g5, v)

    lhs = torch.vdot(chi.reshape(-1), s.M(psi).reshape(-1))
    rhs = torch.vdot(g5m(s.M(g5m(chi))).reshape(-1), psi.reshape(-1))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # the explicit adjoint equals gamma5 M gamma5
    assert torch.abs(s.Mdag(psi) - g5m(s.M(g5m(psi)))).max() < 1e-13
    e, _ = O.to_eo(psi, dims)
    assert torch.abs(s.Mhat_dag(e) - g5m(s.Mhat(g5m(e)))).max() < 1e-13


def test_mhat_dense_adjoint_2x4():
    dims = (2, 2, 2, 2)
    u = torch.as_tensor(synth.random_su3_field(dims, 0.5, 2))
    s = O.CloverSetup(u, 0.12, 1.0)
    a = dense_matrix(s.Mhat, s.Vh)
    ad = dense_matrix(s.Mhat_dag, s.Vh)
    assert torch.abs(ad - a.conj().T).max() < 1e-14


def test_schur_complement_dense_2x4():
    """Mhat equals the Schur complement of the dense full matrix, built from its blocks."""
    dims = (2, 2, 2, 2)
    u = torch.as_tensor(synth.random_su3_field(dims, 0.5, 5))
    s = O.CloverSetup(u, 0.13, 1.0)
    m = dense_full_operator(s)
    ev, od = O.eo_index(dims)
    rows_e = (ev[:, None] * 12 + torch.arange(12)).reshape(-1)
    rows_o = (od[:, None] * 12 + torch.arange(12)).reshape(-1)
    mee = m[rows_e][:, rows_e]
    meo = m[rows_e][:, rows_o]
    moe = m[rows_o][:, rows_e]
    moo = m[rows_o][:, rows_o]
    schur = mee - meo @ torch.linalg.solve(moo, moe)
    a = dense_matrix(s.Mhat, s.Vh)
    assert torch.abs(a - schur).max() < 1e-13


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 2, 2, 6)])
def test_gauge_covariance(dims):
    u = synth.random_su3_field(dims, 0.4, 11)
    om = synth.random_su3_sites(dims, 12)
    ug = synth.gauge_transform(u, om)
    s = O.CloverSetup(torch.as_tensor(u), 0.12, 1.0)
    sg = O.CloverSetup(torch.as_tensor(ug), 0.12, 1.0)
    rng = np.random.default_rng(0)
    lx, ly, lz, lt = dims
    shp = (lt, lz, ly, lx, 4, 3)
    psi = torch.as_tensor(rng.standard_normal(shp) + 1j * rng.standard_normal(shp))
    omt = torch.as_tensor(om)

    def rot(v):
        return torch.einsum("...ab,...sb->...sa", omt, v)

    assert torch.abs(sg.M(rot(psi)) - rot(s.M(psi))).max() < 1e-12
    e, _ = O.to_eo(psi, dims)
    full_e = O.from_eo(e, None, dims)
    got = O.to_eo(O.from_eo(sg.Mhat(O.to_eo(rot(full_e), dims)[0]), None, dims), dims)[0]
    want = O.to_eo(rot(O.from_eo(s.Mhat(e), None, dims)), dims)[0]
    assert torch.abs(got - want).max() < 1e-12
