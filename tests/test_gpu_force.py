"""GPU parity of the action, its gauge gradient G, the su(3) force F and one HMD
step against the oracle; the autograd path against the oracle and against
central finite differences of the GPU action.

Bar: force relative error <= 1e-9 against the FP64 oracle,
with the solves inside at tol 1e-12 (a solve to tol t moves the force by
O(cond * t))."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle.force import force_matrix
from paper_0910_0262_amd import CloverForce, Lattice, capi, synth

from ._gpu_helpers import make_case, max_rel, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), 0.3, 0.12, 1.0, 0),
    ((4, 4, 4, 4), 0.3, 0.12, 0.0, 1),
    ((6, 4, 2, 8), 0.5, 0.124, 1.3, 2),
    ((8, 8, 8, 8), 0.3, 0.125, 1.0, 3),
]
IDS = ["4^4", "4^4-csw0", "6x4x2x8", "8^4"]


@pytest.fixture(scope="module", params=CASES, ids=IDS)
def case(request):
    dims, w, k, c, seed = request.param
    print(f"[force case dims={dims} width={w} kappa={k} csw={c} seed={seed}]", flush=True)
    lat, setup, u, ud = make_case(dims, w, k, c, seed)
    xi = torch.as_tensor(synth.heatbath_xi(dims, seed))
    phi = setup.Mhat_dag(xi)
    S, G, X, _ = O.action_and_gradient(torch.as_tensor(u), k, c, phi, tol=1e-14)
    F = O.project_force(torch.as_tensor(u), G)
    yield dims, lat, u, ud, phi, (S, G, F, X), (k, c)
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_force_parity(case, prec):
    dims, lat, u, ud, phi, (S, G, F, X), _ = case
    S_g, G_g, F_g, X_g, st = lat.action_force(to_dev(phi), prec=prec, tol=1e-12)
    print(f"  {prec}: iters={st['iters']} S={S_g:.10e} oracle S={S:.10e}", flush=True)
    assert abs(S_g - S) < 1e-10 * abs(S)
    assert rel_err(X_g, X) < 1e-10
    assert max_rel(G_g, G) < 1e-9
    assert max_rel(F_g, F) < 1e-9
    # F is the su(3) projection of G: Hermitian traceless coefficients of (i/2) TA(U G^dag)
    Fm = force_matrix(F_g.cpu())
    assert torch.abs(Fm - Fm.conj().transpose(-1, -2)).max() < 1e-12


def test_autograd_backward(case):
    dims, lat, u, ud, phi, (S, G, F, X), (k, c) = case
    U = ud.clone().requires_grad_(True)
    ph = to_dev(phi).requires_grad_(True)
    s = CloverForce.apply(U, ph, lat, "fp64", 1e-12)
    (3.0 * s).backward()
    assert abs(float(s) - S) < 1e-10 * abs(S)
    assert max_rel(U.grad, 3.0 * G) < 1e-9
    assert rel_err(ph.grad, 6.0 * X) < 1e-10


def test_autograd_vs_finite_differences():
    """Central differences (eps = 1e-5) of the GPU action along su(3) generators, 4^4."""
    dims, kappa, csw = (4, 4, 4, 4), 0.12, 1.0
    u = synth.random_su3_field(dims, 0.3, 0)
    lat = Lattice(dims, kappa, csw)
    ud = to_dev(u)
    lat.load_gauge(ud)
    xi = to_dev(synth.heatbath_xi(dims, 0))
    phi = lat.apply("Mhatdag", xi)
    S0, G, F, X, _ = lat.action_force(phi, tol=1e-13)
    lam = O.gell_mann()
    eps = 1e-5
    scale = float(torch.abs(F).max())
    for site, mu, a in [((0, 0, 0, 0), 0, 0), ((1, 2, 3, 0), 3, 4), ((3, 1, 0, 2), 1, 7)]:
        vals = []
        for sgn in (1, -1):
            up = u.copy()
            e = torch.linalg.matrix_exp(1j * sgn * eps * lam[a] / 2).numpy()
            up[site + (mu,)] = e @ u[site + (mu,)]
            lat.load_gauge(to_dev(up))
            # variational action 2 Re phi^dag X - |Mhat X|^2: error quadratic in the residual
            _, _, _, x, _ = lat.action_force(phi, tol=1e-13, want_F=False)
            y = lat.apply("Mhat", x)
            vals.append(float(2.0 * torch.vdot(phi.reshape(-1), x.reshape(-1)).real - torch.vdot(y.reshape(-1), y.reshape(-1)).real))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - float(F[site + (mu, a)])) < 1e-6 * scale
    lat.close()


def test_hmd_step_parity():
    dims, kappa, csw, dt = (4, 4, 4, 4), 0.125, 1.0, 0.02
    u0 = synth.random_su3_field(dims, 0.3, 0)
    p0 = synth.momenta(dims, 0)
    xi = synth.heatbath_xi(dims, 0)
    ref = O.hmd_step(torch.as_tensor(u0), torch.as_tensor(p0), torch.as_tensor(xi), dt, kappa, csw, tol=1e-14)
    lat = Lattice(dims, kappa, csw)
    U = to_dev(u0)
    P = to_dev(p0)
    S, st = lat.hmd_step(U, P, to_dev(xi), dt, prec="fp64", tol=1e-12)
    assert abs(S - ref["S"]) < 1e-10 * abs(ref["S"])
    assert max_rel(U, ref["U"]) < 1e-9
    assert max_rel(P, ref["P"]) < 1e-9
    # unitarity is kept by the exponential update
    uu = U.conj().transpose(-1, -2) @ U
    assert torch.abs(uu - torch.eye(3, dtype=torch.complex128, device="cuda")).max() < 1e-13
    # the same step from the library's own calls in the two-flavour R-algorithm
    # order: phi = Mhat^dag(U_0) xi, links to the midpoint, force there at fixed phi
    lat.load_gauge(to_dev(u0))
    phi0 = lat.apply("Mhatdag", to_dev(xi))
    Uh = to_dev(u0)
    lat.md_trajectory(Uh, to_dev(p0), None, 0.5 * dt, 1, beta=0.0, n_f=0.0)
    lat.load_gauge(Uh)
    _, _, F, _, _ = lat.action_force(phi0, tol=1e-12, want_X=False)
    assert max_rel(P, to_dev(p0) - dt * F) < 1e-10
    lat.close()


def test_hmd_step_parity_16x4():
    """One HMD step at dt = 0.02 on the force workload's lattice (16^4, kappa 0.125, c_sw 1)."""
    dims, kappa, csw, dt = (16, 16, 16, 16), 0.125, 1.0, 0.02
    print("[hmd step 16^4: oracle reference]", flush=True)
    u0 = synth.random_su3_field(dims, 0.3, 4)
    p0 = synth.momenta(dims, 4)
    xi = synth.heatbath_xi(dims, 4)
    ref = O.hmd_step(torch.as_tensor(u0), torch.as_tensor(p0), torch.as_tensor(xi), dt, kappa, csw, tol=1e-13)
    lat = Lattice(dims, kappa, csw)
    for prec in ("fp64", "mixed"):
        U = to_dev(u0)
        P = to_dev(p0)
        S, st = lat.hmd_step(U, P, to_dev(xi), dt, prec=prec, tol=1e-12)
        print(f"  16^4 {prec}: iters={st['iters']} S={S:.12e} oracle {ref['S']:.12e}", flush=True)
        assert abs(S - ref["S"]) < 1e-10 * abs(ref["S"])
        assert max_rel(U, ref["U"]) < 1e-9
        assert max_rel(P, ref["P"]) < 1e-9
    lat.close()


def test_hmd_step_mixed_solve():
    dims, kappa, csw, dt = (8, 8, 8, 8), 0.125, 1.0, 0.02
    u0 = synth.random_su3_field(dims, 0.3, 1)
    p0 = synth.momenta(dims, 1)
    xi = synth.heatbath_xi(dims, 1)
    ref = O.hmd_step(torch.as_tensor(u0), torch.as_tensor(p0), torch.as_tensor(xi), dt, kappa, csw, tol=1e-13)
    lat = Lattice(dims, kappa, csw)
    U = to_dev(u0)
    P = to_dev(p0)
    lat.hmd_step(U, P, to_dev(xi), dt, prec="mixed", tol=1e-12)
    assert max_rel(U, ref["U"]) < 1e-9
    assert max_rel(P, ref["P"]) < 1e-9
    lat.close()


@pytest.fixture(scope="module")
def force16():
    """The force lattice of the benchmark configurations: 16^4, kappa 0.125, c_sw 1, width 0.3."""
    dims, kappa, csw = (16, 16, 16, 16), 0.125, 1.0
    print("[force 16^4: oracle reference]", flush=True)
    lat, setup, u, ud = make_case(dims, 0.3, kappa, csw, 2)
    phi = setup.Mhat_dag(torch.as_tensor(synth.heatbath_xi(dims, 2)))
    S, G, X, _ = O.action_and_gradient(torch.as_tensor(u), kappa, csw, phi, tol=1e-13)
    F = O.project_force(torch.as_tensor(u), G)
    yield lat, phi, (S, G, F, X)
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_force_parity_16x4(force16, prec):
    lat, phi, (S, G, F, X) = force16
    S_g, G_g, F_g, X_g, st = lat.action_force(to_dev(phi), prec=prec, tol=1e-12)
    print(f"  16^4 {prec}: iters={st['iters']}", flush=True)
    assert abs(S_g - S) < 1e-10 * abs(S)
    assert rel_err(X_g, X) < 1e-10
    assert max_rel(G_g, G) < 1e-9
    assert max_rel(F_g, F) < 1e-9


def test_force_directional_fd_full_lattice():
    """32^3 x 64 (the benchmark's lattice, force with the mixed solve inside):
    the library's force against the derivative of the oracle's action along
    U -> exp(i eps sum_a Q^a T^a) U for a random Q on every link (central
    difference, eps = 1e-4; the links moved by the oracle's exponential).  The
    action is evaluated by the oracle in its variational form
    S = 2 Re phi^dag X - |Mhat X|^2 with its own Mhat at the moved links and
    phi = Mhat^dag(U) xi from the oracle; S is stationary in X, so the FP64
    solutions X of the library (tol 1e-12) enter only at second order in
    their error, and the check rests on the oracle's operator.  (The oracle's
    own solve would take many minutes at this size.)"""
    dims, kappa, csw, eps = (32, 32, 32, 64), 0.1255, 1.0, 1e-4
    print("[force 32^3x64: directional finite difference of the oracle's action]", flush=True)
    u0 = torch.as_tensor(synth.random_su3_field(dims, 0.2, 0))
    setup = O.CloverSetup(u0, kappa, csw)
    phi = setup.Mhat_dag(torch.as_tensor(synth.heatbath_xi(dims, 0)))
    del setup
    lat = Lattice(dims, kappa, csw)
    lat.load_gauge(to_dev(u0))
    _, _, F, _, _ = lat.action_force(to_dev(phi), prec="mixed", tol=1e-12, want_X=False)
    Q = torch.as_tensor(synth.momenta(dims, 5))
    analytic = float((F.cpu() * Q).sum())
    del F
    vals = []
    for sgn in (1.0, -1.0):
        U = O.expi_su3(Q, sgn * eps) @ u0
        lat.load_gauge(to_dev(U))
        _, _, _, X, _ = lat.action_force(to_dev(phi), prec="fp64", tol=1e-12, want_F=False)
        X = X.cpu()
        y = O.CloverSetup(U, kappa, csw).Mhat(X)
        vals.append(float(2.0 * torch.vdot(phi.reshape(-1), X.reshape(-1)).real
                          - torch.vdot(y.reshape(-1), y.reshape(-1)).real))
        print(f"  S({sgn * eps:+.0e}) = {vals[-1]:.12e}", flush=True)
    fd = (vals[0] - vals[1]) / (2 * eps)
    print(f"  fd={fd:.9e} analytic={analytic:.9e} rel={abs(fd - analytic) / abs(analytic):.2e}", flush=True)
    assert abs(fd - analytic) < 1e-5 * abs(analytic)
    lat.close()
