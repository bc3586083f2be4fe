"""Pins of the oracle's HMD step: exact reversibility, unitarity, and the dt^3
scaling of the energy violation of one leapfrog step with the pseudofermion held fixed."""
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


def test_hmd_reversibility():
    u0 = torch.as_tensor(synth.random_su3_field(DIMS, 0.3, 0))
    p0 = torch.as_tensor(synth.momenta(DIMS, 0))
    xi = torch.as_tensor(synth.heatbath_xi(DIMS, 0))
    dt = 0.02
    st = O.hmd_step(u0, p0, xi, dt, KAPPA, CSW)
    back = O.hmd_step(st["U"], -st["P"], xi, dt, KAPPA, CSW)
    assert torch.abs(back["U"] - u0).max() < 1e-12
    assert torch.abs(back["P"] + p0).max() < 1e-10


def _leapfrog_fixed_phi(u0, p0, phi, dt):
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
