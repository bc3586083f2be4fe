"""Oracle: one hybrid-molecular-dynamics step of the pseudofermion system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs MILC's su3_rmd, the R algorithm (abstract, section 1), whose
details are in a reference the text does not reproduce.  The oracle takes the
two-flavour reading, where the R algorithm's flavour-dependent time shift of
the pseudofermion refresh vanishes, and performs one position-momentum-
position leapfrog step with the pseudofermion refreshed at the midpoint:

    U_1/2 = exp(i dt/2 P_0) U_0
    phi   = Mhat^dag(U_1/2) xi
    P_1   = P_0 - dt F(U_1/2, phi)
    U_1   = exp(i dt/2 P_1) U_1/2

with P = sum_a P^a T^a and F^a = dS/dw^a (see oracle.force).  The gauge
action is not part of this step.
"""
from __future__ import annotations

import torch

from .core import CloverSetup, gell_mann
from .force import action_and_gradient, project_force
from .solve import _dot


def expi_su3(p_coeff: torch.Tensor, c: float) -> torch.Tensor:
    """exp(i c sum_a P^a T^a) by eigen-decomposition of the Hermitian matrix."""
    h = torch.einsum("...a,aij->...ij", torch.as_tensor(p_coeff).to(torch.complex128), gell_mann() / 2)
    w, v = torch.linalg.eigh(h)
    return (v * torch.exp(1j * c * w).unsqueeze(-2)) @ v.conj().transpose(-1, -2)


def hmd_step(u0, p0, xi_e, dt, kappa, csw, tol=1e-13, t_boundary=-1.0):
    """Returns dict(U=U_1, P=P_1, phi, S, F, U_half)."""
    u0 = torch.as_tensor(u0)
    p0 = torch.as_tensor(p0)
    u_half = expi_su3(p0, dt / 2) @ u0
    setup = CloverSetup(u_half, kappa, csw, t_boundary)
    phi = setup.Mhat_dag(torch.as_tensor(xi_e))
    s, g, _, _ = action_and_gradient(u_half, kappa, csw, phi, tol, t_boundary)
    f = project_force(u_half, g)
    p1 = p0 - dt * f
    u1 = expi_su3(p1, dt / 2) @ u_half
    return {"U": u1, "P": p1, "phi": phi, "S": s, "F": f, "U_half": u_half}


def hamiltonian(u, p, phi_e, kappa, csw, tol=1e-13, t_boundary=-1.0) -> float:
    """H = 1/2 sum (P^a)^2 + S(U, phi)."""
    from .solve import cg

    setup = CloverSetup(torch.as_tensor(u), kappa, csw, t_boundary)
    x = cg(setup.MdagM, phi_e, tol).x
    return 0.5 * float((torch.as_tensor(p) ** 2).sum()) + float(_dot(phi_e, x).real)
