"""Oracle: the rest of the molecular-dynamics action and a multi-step trajectory.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's application evolves dynamical clover fermions with the HMD R
algorithm (abstract, section 1); the actions it integrates are not printed.
Textbook definitions, written out:

* Wilson gauge action  S_g = beta sum_{x, mu<nu} (1 - Re tr U_mu,nu(x) / 3),
  U_mu,nu(x) = U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag.
* Even-odd clover determinant: the Schur complement gives
  det M = det A_oo det Mhat exactly, so with the pseudofermion covering
  det(Mhat^dag Mhat) the remaining two-flavour factor (det A_oo)^2 enters as
  S_det = -2 sum_{x odd} ln det A(x)  (A(x) Hermitian positive definite).
* Force of any part: F^a = dS/dw^a for U -> exp(i w^a T^a) U, obtained from
  the PyTorch-convention gradient G by F^a = Re{ i tr[T^a U G^dag] }.
* Trajectory: n steps of the R algorithm for N_f flavours (Gottlieb, Liu,
  Toussaint, Renken, Sugar, Phys. Rev. D 35 (1987) 2531), with the schedule
  of oracle.hmd.r_step: in each step the links move by (1 - N_f/2) dt/2, the
  pseudofermion is refreshed there from the step's own noise vector, the
  links move on to the midpoint by (N_f/2) dt/2, the momenta take dt times
  the force with the fermion and determinant parts weighted by N_f/2, and
  the links take the last dt/2.  At N_f = 2 the refresh happens at the start
  of the step, which is then a heat-bath of phi and one leapfrog step at
  fixed phi.
* Reunitarisation: Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1).
"""
from __future__ import annotations

import torch

from .core import CloverSetup, clover_matrix, eo_index
from .force import action_and_gradient, project_force
from .hmd import expi_su3, r_step
from .solve import _dot, cg


def _sh(f, mu, n):
    return torch.roll(f, -n, dims=3 - mu)


def plaquettes(u: torch.Tensor) -> dict:
    """U_mu,nu(x) for mu < nu, (Lt, Lz, Ly, Lx, 3, 3) each."""
    out = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            um, un = u[..., mu, :, :], u[..., nu, :, :]
            out[(mu, nu)] = um @ _sh(un, mu, 1) @ _sh(um, nu, 1).conj().transpose(-1, -2) @ un.conj().transpose(-1, -2)
    return out


def gauge_action(u: torch.Tensor, beta: float) -> torch.Tensor:
    """S_g = beta sum (1 - Re tr P / 3) (a 0-dim tensor, differentiable)."""
    s = torch.zeros((), dtype=torch.float64)
    for p in plaquettes(u).values():
        s = s + (1.0 - torch.diagonal(p, dim1=-2, dim2=-1).sum(-1).real / 3.0).sum()
    return beta * s


def clover_det_action(u: torch.Tensor, kappa: float, csw: float) -> torch.Tensor:
    """S_det = -2 sum_{x odd} ln det A(x); A Hermitian positive definite."""
    lt, lz, ly, lx = u.shape[:4]
    a = clover_matrix(u, kappa, csw).reshape(-1, 12, 12)
    _, od = eo_index((lx, ly, lz, lt))
    sign, logdet = torch.linalg.slogdet(a[od])
    return -2.0 * logdet.real.sum()


def gradient(action_fn, u: torch.Tensor) -> torch.Tensor:
    ug = torch.as_tensor(u).detach().clone().requires_grad_(True)
    (g,) = torch.autograd.grad(action_fn(ug), ug)
    return g


def reunitarize(u: torch.Tensor) -> torch.Tensor:
    """Gram-Schmidt on rows 0 and 1, then row 2 = conj(row0 x row1)."""
    a = u[..., 0, :]
    a = a / torch.linalg.norm(a, dim=-1, keepdim=True)
    b = u[..., 1, :]
    b = b - (a.conj() * b).sum(-1, keepdim=True) * a
    b = b / torch.linalg.norm(b, dim=-1, keepdim=True)
    c = torch.linalg.cross(a, b).conj()
    return torch.stack([a, b, c], dim=-2)


def total_force(u, phi_e, kappa, csw, beta, with_det=True, tol=1e-13, t_boundary=-1.0, n_f=2.0):
    """su(3) force of (N_f/2)(S_f + S_det) + S_g and the three action values (unweighted)."""
    u = torch.as_tensor(u)
    wf = n_f / 2.0
    s_f, g_f, _, _ = action_and_gradient(u, kappa, csw, phi_e, tol, t_boundary)
    g = wf * g_f
    parts = {"fermion": s_f, "gauge": 0.0, "det": 0.0}
    if beta != 0.0:
        g = g + gradient(lambda v: gauge_action(v, beta), u)
        parts["gauge"] = float(gauge_action(u, beta))
    if with_det and csw != 0.0:
        g = g + wf * gradient(lambda v: clover_det_action(v, kappa, csw), u)
        parts["det"] = float(clover_det_action(u, kappa, csw))
    return project_force(u, g), parts


def _move(u, p, c):
    return u if c == 0.0 else expi_su3(p, c) @ u


def trajectory(u0, p0, xis, dt, kappa, csw, beta, with_det=True, n_f=2.0, reunit=False, tol=1e-13,
               t_boundary=-1.0):
    """len(xis) R-algorithm steps (oracle.hmd.r_step); step k refreshes phi = Mhat^dag xi_k.

    Returns (U, P, per-step list of the action parts at each midpoint)."""
    actions = []
    state = (torch.as_tensor(u0), torch.as_tensor(p0))

    def move(st, h):
        return _move(st[0], st[1], h), st[1]

    def kick(st, phi, h):
        f, parts = total_force(st[0], phi, kappa, csw, beta, with_det, tol, t_boundary, n_f)
        actions.append(parts)
        return st[0], st[1] - h * f

    for xi in xis:
        def refresh(st, xi=xi):
            return CloverSetup(st[0], kappa, csw, t_boundary).Mhat_dag(torch.as_tensor(xi))

        u, p = r_step(state, dt, n_f, move, refresh, kick)
        state = (reunitarize(u) if reunit else u), p
    return state[0], state[1], actions


def hamiltonian_fixed_phi(u, p, phi_e, kappa, csw, beta, with_det=True, tol=1e-14, t_boundary=-1.0) -> float:
    """1/2 sum P^2 + S_f(phi) + S_g + S_det at fixed phi."""
    u = torch.as_tensor(u)
    setup = CloverSetup(u, kappa, csw, t_boundary)
    x = cg(setup.MdagM, phi_e, tol).x
    h = 0.5 * float((torch.as_tensor(p) ** 2).sum()) + float(_dot(phi_e, x).real)
    if beta != 0.0:
        h += float(gauge_action(u, beta))
    if with_det and csw != 0.0:
        h += float(clover_det_action(u, kappa, csw))
    return h


def leapfrog_fixed_phi(u0, p0, phi_e, dt, n_steps, kappa, csw, beta, with_det=True, tol=1e-14, t_boundary=-1.0):
    """n leapfrog steps with phi held fixed (an HMC-style trajectory), for the dt^2 pin."""
    u, p = torch.as_tensor(u0), torch.as_tensor(p0)
    for _ in range(n_steps):
        u = expi_su3(p, dt / 2) @ u
        f, _ = total_force(u, phi_e, kappa, csw, beta, with_det, tol, t_boundary)
        p = p - dt * f
        u = expi_su3(p, dt / 2) @ u
    return u, p
