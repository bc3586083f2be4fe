"""Pins of the oracle's HMD step: unitarity, the two-flavour (Phi-algorithm)
limit of the R-algorithm step -- a heat-bath of phi at the start of the step,
then one leapfrog step at fixed phi -- and the dt^3 scaling of the energy
violation of one leapfrog step with the pseudofermion held fixed."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.force import project_force
from paper_0910_0262_amd import synth

DIMS = (4, 2, 2, 4)
KAPPA, CSW = 0.12, 1.0


def test_expi_is_su3_and_inverse():
    p = torch.as_tensor(synth.momenta(DIMS, 0))
    e = O.expi_su3(p, 0.37)
    eye = torch.eye(3, dtype=torch.complex128)
    assert torch.abs(e.conj().transpose(-1, -2) @ e - eye).max() < 1e-14
    assert torch.abs(torch.linalg.det(e) - 1).max() < 1e-14
    assert torch.abs(O.expi_su3(-p, 0.37) @ e - eye).max() < 1e-14


def test_hmd_step_is_phi_algorithm_step():
    """At N_f = 2 the noise is drawn at U_0: the step is phi = Mhat^dag(U_0) xi
    followed by one leapfrog step at fixed phi (written out independently here)."""
    u0 = torch.as_tensor(synth.random_su3_field(DIMS, 0.3, 0))
    p0 = torch.as_tensor(synth.momenta(DIMS, 0))
    xi = torch.as_tensor(synth.heatbath_xi(DIMS, 0))
    dt = 0.02
    st = O.hmd_step(u0, p0, xi, dt, KAPPA, CSW, tol=1e-14)
    phi0 = O.CloverSetup(u0, KAPPA, CSW).Mhat_dag(xi)
    assert torch.abs(st["phi"] - phi0).max() < 1e-15 * torch.abs(phi0).max()
    u1, p1 = _leapfrog_fixed_phi(u0, p0, phi0, dt)
    assert torch.abs(st["U"] - u1).max() < 1e-13
    assert torch.abs(st["P"] - p1).max() < 1e-13 * max(1.0, float(torch.abs(p1).max()))
    # the force is taken at the midpoint, not where phi was drawn
    assert torch.abs(st["U_half"] - O.expi_su3(p0, dt / 2) @ u0).max() < 1e-15
    # a refresh at the midpoint (the step with the shift reversed) is a different step
    phi_half = O.CloverSetup(st["U_half"], KAPPA, CSW).Mhat_dag(xi)
    assert torch.abs(phi_half - phi0).max() > 1e-3 * torch.abs(phi0).max()


def test_hmd_step_unitary():
    u0 = torch.as_tensor(synth.random_su3_field(DIMS, 0.3, 2))
    p0 = torch.as_tensor(synth.momenta(DIMS, 2))
    xi = torch.as_tensor(synth.heatbath_xi(DIMS, 2))
    u1 = O.hmd_step(u0, p0, xi, 0.05, KAPPA, CSW)["U"]
    eye = torch.eye(3, dtype=torch.complex128)
    assert torch.abs(u1.conj().transpose(-1, -2) @ u1 - eye).max() < 1e-14
    assert torch.abs(torch.linalg.det(u1) - 1).max() < 1e-14


def _leapfrog_fixed_phi(u0, p0, phi, dt):
    """One position-momentum-position step at fixed phi, written out."""
    uh = O.expi_su3(p0, dt / 2) @ u0
    _, g, _, _ = O.action_and_gradient(uh, KAPPA, CSW, phi, tol=1e-14)
    p1 = p0 - dt * project_force(uh, g)
    return O.expi_su3(p1, dt / 2) @ uh, p1


@pytest.mark.slow
def test_energy_violation_scales_as_dt_cubed():
    u0 = torch.as_tensor(synth.random_su3_field(DIMS, 0.3, 1))
    p0 = torch.as_tensor(synth.momenta(DIMS, 1))
    s = O.CloverSetup(u0, KAPPA, CSW)
    phi = s.Mhat_dag(torch.as_tensor(synth.heatbath_xi(DIMS, 1)))
    h0 = O.hamiltonian(u0, p0, phi, KAPPA, CSW, tol=1e-14)
    dh = []
    for dt in (0.04, 0.02):
        u1, p1 = _leapfrog_fixed_phi(u0, p0, phi, dt)
        dh.append(abs(O.hamiltonian(u1, p1, phi, KAPPA, CSW, tol=1e-14) - h0))
    ratio = dh[0] / dh[1]
    assert 6.0 < ratio < 10.0, (dh, ratio)
