"""Oracle: conjugate gradient on the even-odd normal equations, full solve, dense matrices.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's application (abstract, section 1) solves the clover Dirac
equation inside every molecular-dynamics step; the solver it uses is not
described in the text.  The oracle uses the textbook Hestenes-Stiefel CG on
Mhat^dag Mhat x_e = Mhat^dag bhat, started from x = 0, and stops when
||r_k|| <= tol ||Mhat^dag bhat||.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from .core import CloverSetup, from_eo, to_eo


def _dot(a, b):
    return torch.vdot(a.reshape(-1), b.reshape(-1))


@dataclass
class CGResult:
    x: torch.Tensor
    iters: int
    converged: bool
    rel_res: float  # recomputed ||b - A x|| / ||b||


def cg(apply_a, b: torch.Tensor, tol: float, max_iter: int = 20000, x0=None) -> CGResult:
    """Textbook CG for a Hermitian positive-definite operator ``apply_a``."""
    if x0 is None:
        x = torch.zeros_like(b)
        r = b.clone()
    else:
        x = x0.clone()
        r = b - apply_a(x)
    p = r.clone()
    rr = _dot(r, r).real
    bb = _dot(b, b).real
    stop = tol * tol * bb
    k = 0
    converged = bool(rr <= stop)
    while not converged and k < max_iter:
        ap = apply_a(p)
        alpha = rr / _dot(p, ap).real
        x = x + alpha * p
        r = r - alpha * ap
        rr_new = _dot(r, r).real
        k += 1
        if rr_new <= stop:
            converged = True
            break
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    true_r = b - apply_a(x)
    rel = float(torch.sqrt(_dot(true_r, true_r).real / bb)) if bb > 0 else 0.0
    return CGResult(x, k, converged, rel)


@dataclass
class SolveResult:
    x: torch.Tensor          # full-lattice solution (Lt, Lz, Ly, Lx, 4, 3)
    iters: int
    converged: bool
    normal_rel_res: float    # ||Mhat^dag bhat - Mhat^dag Mhat x_e|| / ||Mhat^dag bhat||
    true_rel_res: float      # ||b - M x|| / ||b|| on the full lattice


def solve_full(setup: CloverSetup, b: torch.Tensor, tol: float, max_iter: int = 20000) -> SolveResult:
    """Solve M x = b on the full lattice by even-odd preconditioning.

    bhat = b_e + kappa H_eo A_oo^{-1} b_o; CG on Mhat^dag Mhat x_e = Mhat^dag bhat;
    x_o = A_oo^{-1} (b_o + kappa H_oe x_e)."""
    b_e, b_o = to_eo(b, setup.dims)
    bhat = setup.prepare(b_e, b_o)
    rhs = setup.Mhat_dag(bhat)
    res = cg(setup.MdagM, rhs, tol, max_iter)
    x_o = setup.reconstruct(res.x, b_o)
    x = from_eo(res.x, x_o, setup.dims)
    r = b - setup.M(x)
    true_rel = float(torch.sqrt(_dot(r, r).real / _dot(b, b).real))
    return SolveResult(x, res.iters, res.converged, res.rel_res, true_rel)


def dense_matrix(apply_op, n_sites: int, chunk: int = 512) -> torch.Tensor:
    """Dense matrix of a linear map on (n_sites, 4, 3) vectors, by applying it to unit vectors.

    Column j is op(e_j); rows and columns use the flattening (site, spin, colour)."""
    n = n_sites * 12
    cols = []
    for start in range(0, n, chunk):
        stop = min(n, start + chunk)
        basis = torch.zeros(stop - start, n, dtype=torch.complex128)
        basis[torch.arange(stop - start), torch.arange(start, stop)] = 1.0
        out = apply_op(basis.reshape(stop - start, n_sites, 4, 3))
        cols.append(out.reshape(stop - start, n))
    return torch.cat(cols, 0).T.contiguous()


def dense_full_operator(setup: CloverSetup, which: str = "M", chunk: int = 512) -> torch.Tensor:
    """Dense full-lattice M (or M^dag, H) as a (12V, 12V) matrix, lexicographic site order."""
    lx, ly, lz, lt = setup.dims
    op = {"M": setup.M, "Mdag": setup.Mdag, "H": setup.H}[which]

    def apply(v):
        return op(v.reshape(v.shape[0], lt, lz, ly, lx, 4, 3)).reshape(v.shape[0], -1, 4, 3)

    return dense_matrix(apply, setup.V, chunk)
