"""Each test plants a plausible mistake in the oracle (on the CPU, by monkeypatching)
and checks that at least one of the pins fails.  This shows the pins constrain
the oracle: a dropped sign, a swapped projector, a reversed leaf or a
transposed gradient does not slip through."""
import pytest
import torch

import oracle as O
import oracle.core as core
import oracle.force as force
from paper_0910_0262_amd import synth

from . import test_oracle_clover as tc
from . import test_oracle_operator as to
from . import test_oracle_force as tf


def test_swapped_projectors_fail_plane_wave(monkeypatch):
    g = core.gammas()
    monkeypatch.setattr(core, "gammas", lambda: -g)
    with pytest.raises(AssertionError):
        to.test_plane_wave_free((4, 4, 4, 4))


def test_missing_time_boundary_sign_fails_spectrum(monkeypatch):
    orig = core.hop
    monkeypatch.setattr(core, "hop", lambda u, psi, t_boundary=-1.0, dagger=False: orig(u, psi, 1.0, dagger))
    with pytest.raises(AssertionError):
        to.test_free_field_spectrum_M_2x4(-1)


def test_backward_hop_without_dagger_fails_gamma5_hermiticity(monkeypatch):
    monkeypatch.setattr(core, "hop", _hop_no_dagger)
    with pytest.raises(AssertionError):
        to.test_gamma5_hermiticity((4, 4, 4, 4), 0.3, 0.12)


def _hop_no_dagger(u, psi, t_boundary=-1.0, dagger=False):
    """The hopping term with U_mu(x-mu) used where U_mu(x-mu)^dag belongs."""
    lt = u.shape[0]
    g = core.gammas()
    one = torch.eye(4, dtype=torch.complex128)
    sgn = -1.0 if dagger else 1.0
    out = torch.zeros_like(psi)
    for mu in range(4):
        ax = -3 - mu
        umu = u[..., mu, :, :]
        fwd = torch.roll(psi, -1, dims=ax)
        bwd = torch.roll(torch.einsum("...ab,...sb->...sa", umu, psi), 1, dims=ax)
        if mu == 3:
            ef = torch.ones(lt, dtype=torch.float64)
            ef[-1] = t_boundary
            eb = torch.ones(lt, dtype=torch.float64)
            eb[0] = t_boundary
            fwd = fwd * ef.view(lt, 1, 1, 1, 1, 1)
            bwd = bwd * eb.view(lt, 1, 1, 1, 1, 1)
        fwd = torch.einsum("...ab,...sb->...sa", umu, fwd)
        out = out + torch.einsum("st,...tb->...sb", one - sgn * g[mu], fwd)
        out = out + torch.einsum("st,...tb->...sb", one + sgn * g[mu], bwd)
    return out


def test_reversed_leaf_fails_abelian_flux(monkeypatch):
    def bad_leaves(u, mu, nu):
        um = u[..., mu, :, :]
        un = u[..., nu, :, :]
        sh, dag = core._sh, core._dag
        q = um @ sh(un, mu, 1) @ dag(sh(um, nu, 1)) @ dag(un)
        q = q + dag(un @ dag(sh(sh(um, mu, -1), nu, 1)) @ dag(sh(un, mu, -1)) @ sh(um, mu, -1))  # reversed
        q = q + dag(sh(um, mu, -1)) @ dag(sh(sh(un, mu, -1), nu, -1)) @ sh(sh(um, mu, -1), nu, -1) @ sh(un, nu, -1)
        q = q + dag(sh(un, nu, -1)) @ sh(um, nu, -1) @ sh(sh(un, mu, 1), nu, -1) @ dag(um)
        return q

    monkeypatch.setattr(core, "clover_leaves", bad_leaves)
    with pytest.raises(AssertionError):
        tc.test_abelian_flux_closed_form((4, 4, 2, 2), 1)


def test_dropped_traceless_projection_fails_u1_flux(monkeypatch):
    def no_trace_removal(u):
        out = {}
        for mu in range(4):
            for nu in range(mu + 1, 4):
                q = core.clover_leaves(u, mu, nu)
                out[(mu, nu)] = (q - core._dag(q)) / 8j
        return out

    monkeypatch.setattr(core, "clover_field_strength", no_trace_removal)
    with pytest.raises(AssertionError):
        tc.test_abelian_flux_u1_embedding_traceless_projection()


def test_transposed_gradient_fails_fd(monkeypatch):
    orig = force.gradient_from_solution
    monkeypatch.setattr(force, "gradient_from_solution", lambda *a, **k: orig(*a, **k).transpose(-1, -2))
    u = torch.as_tensor(synth.random_su3_field(tf.DIMS, 0.3, 0))
    with pytest.raises(AssertionError):
        tf.test_gradient_vs_fd_unconstrained(u)


def test_wrong_force_sign_fails_fd(monkeypatch):
    orig = force.gradient_from_solution
    monkeypatch.setattr(force, "gradient_from_solution", lambda *a, **k: -orig(*a, **k))
    u = torch.as_tensor(synth.random_su3_field(tf.DIMS, 0.3, 0))
    with pytest.raises(AssertionError):
        tf.test_force_vs_fd_generators(u, 1.0)


# ---------------------------------------------------------------- gauge action, determinant, reunitarisation
from oracle import md  # noqa: E402

from . import test_oracle_md as tm  # noqa: E402


def test_open_plaquette_fails_coordinate_loop(monkeypatch):
    def bad_plaquettes(u):
        out = {}
        for mu in range(4):
            for nu in range(mu + 1, 4):
                um, un = u[..., mu, :, :], u[..., nu, :, :]
                # U_nu taken at x - mu instead of x + mu
                out[(mu, nu)] = um @ md._sh(un, mu, -1) @ md._sh(um, nu, 1).conj().transpose(-1, -2) @ \
                    un.conj().transpose(-1, -2)
        return out

    monkeypatch.setattr(md, "plaquettes", bad_plaquettes)
    with pytest.raises(AssertionError):
        tm.test_gauge_action_coordinate_loop()


def test_one_flavour_determinant_fails_flux_closed_form(monkeypatch):
    orig = md.clover_det_action
    monkeypatch.setattr(md, "clover_det_action", lambda u, k, c: 0.5 * orig(u, k, c))
    with pytest.raises(AssertionError):
        tm.test_clover_det_abelian_flux_closed_form(1)


@pytest.mark.slow
def test_even_site_determinant_fails_two_flavour_identity(monkeypatch):
    def det_even(u, kappa, csw):
        lt, lz, ly, lx = u.shape[:4]
        a = core.clover_matrix(u, kappa, csw).reshape(-1, 12, 12)
        ev, _ = core.eo_index((lx, ly, lz, lt))
        return -2.0 * torch.linalg.slogdet(a[ev])[1].sum()

    monkeypatch.setattr(md, "clover_det_action", det_even)
    with pytest.raises(AssertionError):
        tm.test_two_flavour_identity_full_determinant()


def test_reunitarize_without_conjugate_fails(monkeypatch):
    def bad(u):
        a = u[..., 0, :] / torch.linalg.norm(u[..., 0, :], dim=-1, keepdim=True)
        b = u[..., 1, :] - (a.conj() * u[..., 1, :]).sum(-1, keepdim=True) * a
        b = b / torch.linalg.norm(b, dim=-1, keepdim=True)
        return torch.stack([a, b, torch.linalg.cross(a, b)], dim=-2)

    monkeypatch.setattr(md, "reunitarize", bad)
    with pytest.raises(AssertionError):
        tm.test_reunitarize()
