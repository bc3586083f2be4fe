"""Oracle: one hybrid-molecular-dynamics step of the pseudofermion system.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper runs MILC's su3_rmd, the R algorithm (abstract, section 1), whose
steps are in a reference the text does not reproduce: Gottlieb, Liu,
Toussaint, Renken and Sugar, Phys. Rev. D 35 (1987) 2531.  In that
algorithm a pseudofermion field carries n flavours (n = 2 for Wilson-type
fermions: phi^dag (M^dag M)^-1 phi) and is redrawn, from fresh Gaussian
noise, every step.  For N_f flavours the fermion force is weighted by N_f/n,
and the noise is drawn (N_f/n) dt/2 before the point where the force is
evaluated, i.e. at t + (1 - N_f/n) dt/2 for a force at the midpoint
t + dt/2.  The correlation between that earlier noise and the momentum
cancels the O(dt) heating which the noisy force would otherwise cause, so
observables carry O(dt^2) errors.  At N_f = n the noise is drawn at the
start of the step and the step is a heat-bath of phi followed by one
position-momentum-position leapfrog step at fixed phi (the Phi algorithm of
the same paper).

``r_step`` is that schedule, written once over three callables so that the
lattice step below, the trajectory of ``oracle.md`` and a one-variable model
in the tests all run the same ordering.  ``hmd_step`` is the N_f = 2 step
with the fermion action alone:

    phi   = Mhat^dag(U_0) xi
    U_1/2 = exp(i dt/2 P_0) U_0
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


def r_step(state, dt, n_f, move, refresh, kick, n_per_field=2.0):
    """One R-algorithm step for N_f flavours (n_per_field flavours per pseudofermion field).

    move(state, h)         -> state with the positions advanced by h times the momenta
    refresh(state)         -> the pseudofermion field drawn at these positions
    kick(state, phi, dt)   -> state with the momenta moved by -dt times the force
                              (fermion part weighted N_f/n_per_field) at phi
    The positions reach the force point t + dt/2 in two moves with the refresh
    between them: (1 - N_f/n) dt/2 before it, (N_f/n) dt/2 after.
    """
    w = n_f / n_per_field
    state = move(state, (1.0 - w) * dt / 2)
    phi = refresh(state)
    state = move(state, w * dt / 2)
    state = kick(state, phi, dt)
    return move(state, dt / 2)


def hmd_step(u0, p0, xi_e, dt, kappa, csw, tol=1e-13, t_boundary=-1.0):
    """Returns dict(U=U_1, P=P_1, phi, S, F, U_half): r_step at N_f = 2, fermion action only."""
    out = {}

    def move(st, h):
        u, p = st
        return (u if h == 0.0 else expi_su3(p, h) @ u), p

    def refresh(st):
        return CloverSetup(st[0], kappa, csw, t_boundary).Mhat_dag(torch.as_tensor(xi_e))

    def kick(st, phi, h):
        u, p = st
        s, g, _, _ = action_and_gradient(u, kappa, csw, phi, tol, t_boundary)
        f = project_force(u, g)
        out.update(phi=phi, S=s, F=f, U_half=u)
        return u, p - h * f

    u1, p1 = r_step((torch.as_tensor(u0), torch.as_tensor(p0)), dt, 2.0, move, refresh, kick)
    out.update(U=u1, P=p1)
    return out


def hamiltonian(u, p, phi_e, kappa, csw, tol=1e-13, t_boundary=-1.0) -> float:
    """H = 1/2 sum (P^a)^2 + S(U, phi)."""
    from .solve import cg

    setup = CloverSetup(torch.as_tensor(u), kappa, csw, t_boundary)
    x = cg(setup.MdagM, phi_e, tol).x
    return 0.5 * float((torch.as_tensor(p) ** 2).sum()) + float(_dot(phi_e, x).real)
