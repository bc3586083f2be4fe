"""Pin of the R-algorithm step schedule (oracle.hmd.r_step) on a one-variable model.

Gottlieb, Liu, Toussaint, Renken and Sugar (Phys. Rev. D 35 (1987) 2531)
draw the pseudofermion noise (N_f/n) dt/2 before the force point so that its
correlation with the momenta cancels the heating of the noisy force, leaving
O(dt^2) errors in observables.  The model keeps exactly that structure:

* position q, momentum p, gauge action q^2/2;
* a 1x1 "fermion matrix" m(q) = sqrt(1 + a q^2), n = 2 flavours per complex
  pseudofermion: target density exp(-q^2/2) (1 + a q^2)^(N_f/2);
* phi = m(q_s) xi with xi complex Gaussian, E|xi|^2 = 1, drawn where r_step
  calls refresh; S_pf = |phi|^2 / m(q)^2, weighted N_f/2 in the force.

If one step moves the equilibrium measure rho(q, p) ~ exp(-p^2/2) target(q)
by O(dt^k), observables averaged over long runs carry O(dt^(k-1)) errors.
The expectation over rho and the noise of a function of the state after one
step is evaluated exactly up to quadrature error by tensor-product Gauss
rules (Hermite in q and p, Laguerre in |xi|^2, which is Exp(1) for a complex
Gaussian), so the pin is deterministic.  The kinetic energy is where the
heating shows: E[p'^2] - E[p^2] falls as dt^2 per step (an O(dt) bias) when
the noise is drawn at the force point, and at least as dt^3 with the R
algorithm's shift.  At N_f = 1 the two orders coincide, so N_f = 2 and 3 are
the cases that discriminate.
"""
import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss
from numpy.polynomial.laguerre import laggauss
from scipy import integrate

from oracle import hmd

A = 2.0


def _rules(n_f, a=A):
    xq, wq = hermegauss(120)
    wq = wq * (1.0 + a * xq * xq) ** (n_f / 2)
    xp, wp = hermegauss(60)
    xe, we = laggauss(60)
    q, p, e = np.meshgrid(xq, xp, xe, indexing="ij")
    w = (wq / wq.sum())[:, None, None] * (wp / wp.sum())[None, :, None] * (we / we.sum())[None, None, :]
    return q, p, e, w


def _one_step(q, p, e, dt, n_f, a=A):
    """The model's callables driven through oracle.hmd.r_step (looked up at call time)."""
    wf = n_f / 2.0

    def move(st, h):
        return st[0] + h * st[1], st[1]

    def refresh(st):
        # |phi|^2 = m(q)^2 |xi|^2; the phase of xi does not enter
        return (1.0 + a * st[0] ** 2) * e

    def kick(st, phi2, h):
        qq, pp = st
        m2 = 1.0 + a * qq * qq
        force = qq + wf * (-phi2 * 2.0 * a * qq / m2 ** 2)
        return qq, pp - h * force

    return hmd.r_step((q, p), dt, n_f, move, refresh, kick)


def _kinetic_drift(n_f, dt):
    q, p, e, w = _rules(n_f)
    q1, p1 = _one_step(q, p, e, dt, n_f)
    return float((w * (p1 * p1 - p * p)).sum())


def test_quadrature_reproduces_the_target():
    for n_f in (2, 3):
        q, p, e, w = _rules(n_f)
        dens = lambda x: np.exp(-x * x / 2) * (1 + A * x * x) ** (n_f / 2)
        z = integrate.quad(dens, -np.inf, np.inf)[0]
        q2 = integrate.quad(lambda x: x * x * dens(x), -np.inf, np.inf)[0] / z
        # (1 + a q^2)^(3/2) is not a polynomial: the Hermite rule is then accurate, not exact
        assert abs(float((w * q * q).sum()) - q2) < 1e-8
        assert abs(float((w * p * p).sum()) - 1.0) < 1e-12
        assert abs(float((w * e).sum()) - 1.0) < 1e-12
        assert _kinetic_drift(n_f, 0.0) == 0.0


@pytest.mark.parametrize("n_f", [2.0, 3.0])
def test_r_step_heating_cancels(n_f):
    d = [_kinetic_drift(n_f, dt) for dt in (0.1, 0.05, 0.025)]
    ratios = [d[i] / d[i + 1] for i in range(2)]
    # O(dt^3) or better per step: at least 8x per halving (O(dt^2) would give 4x)
    assert all(r > 7.0 for r in ratios), (d, ratios)


def test_noise_at_the_force_point_heats():
    """The reversed schedule (noise drawn (N_f/2) dt/2 into the step) heats as dt^2 per
    step; the pin above tells the two apart."""
    def reversed_step(state, dt, n_f, move, refresh, kick, n_per_field=2.0):
        w = n_f / n_per_field
        state = move(state, w * dt / 2)
        phi = refresh(state)
        state = move(state, (1.0 - w) * dt / 2)
        state = kick(state, phi, dt)
        return move(state, dt / 2)

    orig = hmd.r_step
    hmd.r_step = reversed_step
    try:
        for n_f in (2.0, 3.0):
            with pytest.raises(AssertionError):
                test_r_step_heating_cancels(n_f)
            d = [_kinetic_drift(n_f, dt) for dt in (0.1, 0.05)]
            assert 3.5 < d[0] / d[1] < 4.5
    finally:
        hmd.r_step = orig
