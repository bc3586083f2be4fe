"""Pins of the oracle's even-odd solve: dense LU solves of the full system on 2^4 and 4^4,
the full-system residual, and the free-field iteration bound of CG."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.solve import dense_full_operator, dense_matrix
from paper_0910_0262_amd import synth


@pytest.mark.parametrize("dims,width,kappa,seed", [((2, 2, 2, 2), 0.3, 0.12, 0), ((2, 2, 2, 2), 0.5, 0.13, 1)])
def test_solve_matches_dense_2x4(dims, width, kappa, seed):
    u = torch.as_tensor(synth.random_su3_field(dims, width, seed))
    s = O.CloverSetup(u, kappa, 1.0)
    b = torch.as_tensor(synth.gaussian_source(dims, seed, 0))
    res = O.solve_full(s, b, 1e-13)
    assert res.converged
    m = dense_full_operator(s)
    x = torch.linalg.solve(m, b.reshape(-1)).reshape(b.shape)
    err = torch.linalg.norm(res.x - x) / torch.linalg.norm(x)
    assert err < 1e-11
    assert res.true_rel_res < 1e-12


@pytest.mark.slow
def test_solve_matches_dense_4x4():
    dims = (4, 4, 4, 4)
    u = torch.as_tensor(synth.random_su3_field(dims, 0.3, 0))
    s = O.CloverSetup(u, 0.12, 1.0)
    b = torch.as_tensor(synth.gaussian_source(dims, 0, 0))
    res = O.solve_full(s, b, 1e-12)
    m = dense_full_operator(s)
    x = torch.linalg.solve(m, b.reshape(-1)).reshape(b.shape)
    err = float(torch.linalg.norm(res.x - x) / torch.linalg.norm(x))
    assert err < 1e-10
    assert res.true_rel_res < 1e-11


def test_normal_equation_solution_vs_dense_mhat():
    dims = (2, 2, 2, 4)
    u = torch.as_tensor(synth.random_su3_field(dims, 0.3, 3))
    s = O.CloverSetup(u, 0.125, 1.0)
    b = torch.as_tensor(synth.gaussian_source(dims, 3, 0))
    b_e, b_o = O.to_eo(b, dims)
    bhat = s.prepare(b_e, b_o)
    mh = dense_matrix(s.Mhat, s.Vh)
    x_e = torch.linalg.solve(mh, bhat.reshape(-1)).reshape(bhat.shape)
    res = O.cg(s.MdagM, s.Mhat_dag(bhat), 1e-13)
    assert torch.linalg.norm(res.x - x_e) / torch.linalg.norm(x_e) < 1e-11


def test_cg_iterations_free_field_bound():
    """CG on a normal operator with spectrum in [lmin, lmax] needs at most
    ~ 0.5 sqrt(cond) ln(2/tol) iterations; the free-field Mhat^dag Mhat spectrum is known."""
    dims = (4, 4, 4, 4)
    kappa = 0.12
    s = O.CloverSetup(torch.as_tensor(synth.unit_gauge(dims)), kappa, 1.0)
    b = torch.as_tensor(synth.gaussian_source(dims, 0, 0))
    b_e, _ = O.to_eo(b, dims)
    res = O.cg(s.MdagM, b_e, 1e-10)
    lam = []
    for nx in range(4):
        for ny in range(4):
            for nz in range(4):
                for nt in range(4):
                    p = [np.pi * nx / 2, np.pi * ny / 2, np.pi * nz / 2, (2 * nt + 1) * np.pi / 4]
                    c = 2 * sum(np.cos(q) for q in p)
                    sn = 2 * np.sqrt(sum(np.sin(q) ** 2 for q in p))
                    lam.append(abs(1 - kappa ** 2 * (c - 1j * sn) ** 2) ** 2)
    cond = max(lam) / min(lam)
    bound = 0.5 * np.sqrt(cond) * np.log(2 / 1e-10) + 1
    assert res.converged and res.iters <= bound
    assert res.rel_res < 2e-10


def test_enoconv_zero_mode():
    """U = 1, periodic in all directions, kappa = 1/8: the p = 0 mode has M(0) = 1 - 8 kappa = 0."""
    dims = (2, 2, 2, 2)
    s = O.CloverSetup(torch.as_tensor(synth.unit_gauge(dims)), 0.125, 1.0, t_boundary=1.0)
    b = torch.ones((2, 2, 2, 2, 4, 3), dtype=torch.complex128)
    b_e, _ = O.to_eo(b, dims)
    assert torch.abs(s.Mhat(b_e)).max() < 1e-15
