"""Oracle: pseudofermion action S = phi^dag (Mhat^dag Mhat)^{-1} phi and its gauge derivative.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The fermion force drives the R algorithm's molecular-dynamics update
(abstract, section 1 of the paper); the paper gives no formula for it.  The
oracle computes the derivative of S by its definition:

    X = (Mhat^dag Mhat)^{-1} phi,   Y = Mhat X,
    dS = -X^dag d(Mhat^dag Mhat) X = -2 Re[ Y^dag (dMhat) X ],

so with X and Y held fixed, dS/dU is -2 times the gradient of the real
scalar Re[Y^dag Mhat(U) X], which autograd evaluates through the oracle's own
operator (hopping term, clover leaves, 12x12 inverse).  The identity is exact
for the exact solution X.

Gradient convention: G = dS/dRe(U) + i dS/dIm(U) per matrix element (the
PyTorch convention for a real function of complex inputs), so a first-order
change of S is dS = Re sum conj(G) dU.

su(3) force: with U_mu(x) -> exp(i w^a T^a) U_mu(x), T^a = lambda^a / 2,
F^a = dS/dw^a = Re{ i tr[ T^a U G^dag ] }.
"""
from __future__ import annotations

import torch

from .core import CloverSetup, gell_mann
from .solve import cg, _dot


def action(setup: CloverSetup, phi_e: torch.Tensor, tol: float = 1e-13):
    """S = Re phi^dag X with X from CG; returns (S, X, iterations)."""
    res = cg(setup.MdagM, phi_e, tol)
    return float(_dot(phi_e, res.x).real), res.x, res.iters


def action_variational(setup: CloverSetup, phi_e: torch.Tensor, tol: float = 1e-12) -> float:
    """S = 2 Re phi^dag X - X^dag Mhat^dag Mhat X; its error is quadratic in the CG residual."""
    x = cg(setup.MdagM, phi_e, tol).x
    y = setup.Mhat(x)
    return float(2.0 * _dot(phi_e, x).real - _dot(y, y).real)


def gradient_from_solution(u, kappa, csw, x_e, t_boundary=-1.0):
    """G = dS/dU for S = phi^dag (Mhat^dag Mhat)^{-1} phi, given the solution X (fixed)."""
    u = torch.as_tensor(u).detach()
    with torch.no_grad():
        y = CloverSetup(u, kappa, csw, t_boundary).Mhat(x_e)
    ug = u.clone().requires_grad_(True)
    s = CloverSetup(ug, kappa, csw, t_boundary)
    f = _dot(y.detach(), s.Mhat(x_e.detach())).real
    (g,) = torch.autograd.grad(f, ug)
    return -2.0 * g


def action_and_gradient(u, kappa, csw, phi_e, tol: float = 1e-13, t_boundary=-1.0):
    """Returns (S, G, X, iters): action, PyTorch-convention gradient dS/dU, solution, CG iterations."""
    u = torch.as_tensor(u)
    setup = CloverSetup(u, kappa, csw, t_boundary)
    s, x, iters = action(setup, phi_e, tol)
    g = gradient_from_solution(u, kappa, csw, x, t_boundary)
    return s, g, x, iters


def project_force(u, g) -> torch.Tensor:
    """F^a_mu(x) = Re{ i tr[ T^a U_mu(x) G_mu(x)^dag ] }, shape (Lt, Lz, Ly, Lx, 4, 8)."""
    u = torch.as_tensor(u)
    w = u @ g.conj().transpose(-1, -2)
    t = gell_mann() / 2
    return torch.einsum("aij,...ji->...a", t, 1j * w).real


def force_matrix(f_coeff: torch.Tensor) -> torch.Tensor:
    """sum_a F^a T^a: Hermitian traceless 3x3 per link."""
    return torch.einsum("...a,aij->...ij", f_coeff.to(torch.complex128), gell_mann() / 2)
