"""GPU parity of the even-odd solve (FP64 and mixed precision) against the oracle.

Bar: relative solution error <= 1e-10 against the oracle's
FP64 solution, both solved to tol 1e-12 (the solution error can reach
cond(Mhat^dag Mhat) * tol); the true full-lattice residual is checked too."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_0910_0262_amd import Lattice, QCDError, capi, synth

from ._gpu_helpers import make_case, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), 0.3, 0.12, 1.0, 0),
    ((10, 6, 4, 6), 0.5, 0.124, 1.0, 1),
    ((8, 8, 16, 16), 0.5, 0.124, 1.0, 0),
]
IDS = ["4^4", "10x6x4x6", "8x8x16x16"]


@pytest.fixture(scope="module", params=CASES, ids=IDS)
def case(request):
    dims, w, k, c, seed = request.param
    print(f"[solve case dims={dims} width={w} kappa={k} seed={seed}]", flush=True)
    lat, setup, u, ud = make_case(dims, w, k, c, seed)
    b = synth.gaussian_source(dims, seed, 0)
    ref = O.solve_full(setup, torch.as_tensor(b), 1e-13)
    assert ref.converged
    yield dims, lat, setup, b, ref
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_solve_parity(case, prec):
    dims, lat, setup, b, ref = case
    x, st = lat.solve(to_dev(b), prec=prec, tol=1e-12)
    print(f"  {prec}: iters={st['iters']} ru={st['reliable_updates']} true={st['true_rel_res']:.2e}", flush=True)
    assert st["converged"] == 1
    assert rel_err(x, ref.x) < 1e-10
    assert st["true_rel_res"] < 1e-10
    if prec == "mixed":
        # twelve decades at delta 0.1: the FP64 residual is recomputed many times
        assert st["reliable_updates"] >= 5
        assert st["restarts"] == 0
    # the oracle's operator applied to the GPU solution
    r = torch.as_tensor(b) - setup.M(x.cpu())
    assert float(torch.linalg.norm(r) / torch.linalg.norm(torch.as_tensor(b))) < 1e-10


def test_solve_deterministic(case):
    dims, lat, setup, b, ref = case
    x1, s1 = lat.solve(to_dev(b), prec="fp64", tol=1e-10)
    x2, s2 = lat.solve(to_dev(b), prec="fp64", tol=1e-10)
    assert torch.equal(x1, x2) and s1["iters"] == s2["iters"]
    m1, _ = lat.solve(to_dev(b), prec="mixed", tol=1e-10)
    m2, _ = lat.solve(to_dev(b), prec="mixed", tol=1e-10)
    assert torch.equal(m1, m2)


def test_graph_replay_matches_direct_launches(case):
    """Each CG iteration replayed from a captured HIP graph gives bit-identical
    solutions to launching its kernels one by one; several solves in a row, with
    other eager work (operator applications, synchronisations) in between."""
    dims, lat, setup, b, ref = case
    bd = to_dev(b)
    psi = to_dev(np.ones((setup.Vh, 4, 3), complex))
    for prec in ("fp64", "mixed"):
        lat.set_option(capi.QCD_OPT_GRAPH, 0)
        x0, s0 = lat.solve(bd, prec=prec, tol=1e-10)
        lat.set_option(capi.QCD_OPT_GRAPH, 1)
        for rep in range(3):
            lat.apply("MdagM", psi)
            torch.cuda.synchronize()
            x1, s1 = lat.solve(bd, prec=prec, tol=1e-10)
            assert torch.equal(x1, x0), (prec, rep)
            assert s1["iters"] == s0["iters"] and s1["reliable_updates"] == s0["reliable_updates"]


@pytest.mark.parametrize("clover_bits", [16, 32])
def test_mixed_clover_storage_solve(case, clover_bits):
    dims, lat, setup, b, ref = case
    lat.set_option(capi.QCD_OPT_MIXED_CLOVER, clover_bits)
    x, st = lat.solve(to_dev(b), prec="mixed", tol=1e-12)
    lat.set_option(capi.QCD_OPT_MIXED_CLOVER, 16)
    assert st["converged"] == 1 and rel_err(x, ref.x) < 1e-10


def test_solve_default_tolerance_meets_target(case):
    dims, lat, setup, b, ref = case
    for prec in ("fp64", "mixed"):
        x, st = lat.solve(to_dev(b), prec=prec, tol=1e-10)
        assert st["converged"] == 1 and st["normal_rel_res"] <= 1e-10
        assert rel_err(x, ref.x) < 1e-8


def test_enoconv_returns_last_iterate():
    """A cap of a few iterations cannot reach tol: QCD_ENOCONV, with the last iterate and stats written."""
    dims = (4, 4, 4, 4)
    lat, setup, u, ud = make_case(dims, 0.3, 0.12, 1.0, 0)
    b = to_dev(synth.gaussian_source(dims, 0, 0))
    for prec in ("fp64", "mixed"):
        x, st = lat.solve(b, prec=prec, tol=1e-12, max_iter=5, raise_on_noconv=False)
        assert st["status"] == "QCD_ENOCONV" and st["converged"] == 0
        assert 5 <= st["iters"] <= 6 and torch.isfinite(x).all()
        assert 1e-12 < st["normal_rel_res"] < 1.0
        with pytest.raises(QCDError) as e:
            lat.solve(b, prec=prec, tol=1e-12, max_iter=3)
        assert e.value.code == capi.QCD_ENOCONV
    lat.close()


def test_zero_mode_consistent_normal_equations():
    """U = 1, periodic time, kappa = 1/8: the constant mode is an exact zero mode of M.
    CG on the normal equations still converges (the right-hand side Mhat^dag bhat is
    orthogonal to the null space), while the true residual ||b - M x|| cannot vanish."""
    dims = (4, 4, 4, 4)
    lat = Lattice(dims, 0.125, 1.0, t_boundary=1)
    lat.load_gauge(to_dev(synth.unit_gauge(dims)))
    b = to_dev(synth.gaussian_source(dims, 0, 0) + 1.0)
    x, st = lat.solve(b, prec="fp64", tol=1e-10, max_iter=2000, raise_on_noconv=False)
    assert st["converged"] == 1
    assert st["true_rel_res"] > 1e-3
    lat.close()


def test_enan_on_nonfinite_source():
    dims = (4, 4, 4, 4)
    lat, setup, u, ud = make_case(dims, 0.3, 0.12, 1.0, 0)
    b = synth.gaussian_source(dims, 0, 0)
    b[1, 2, 3, 1, 2, 1] = np.nan
    for prec in ("fp64", "mixed"):
        with pytest.raises(QCDError) as e:
            lat.solve(to_dev(b), prec=prec)
        assert e.value.code == capi.QCD_ENAN
    lat.close()


def test_estate_before_load():
    lat = Lattice((4, 4, 4, 4), 0.12, 1.0)
    with pytest.raises(QCDError) as e:
        lat.apply("Mhat", torch.zeros((128, 4, 3), dtype=torch.complex128, device="cuda"))
    assert e.value.code == capi.QCD_ESTATE
    lat.close()


def test_zero_source():
    dims = (4, 4, 4, 4)
    lat, setup, u, ud = make_case(dims, 0.3, 0.12, 1.0, 0)
    for prec in ("fp64", "mixed"):
        x, st = lat.solve(torch.zeros((4, 4, 4, 4, 4, 3), dtype=torch.complex128, device="cuda"), prec=prec)
        assert torch.count_nonzero(x) == 0 and st["iters"] == 0
    lat.close()


@pytest.mark.parametrize("cycle", [1, 3, 4])
def test_mixed_fallback_to_fp64(case, cycle):
    """QCD_OPT_MIXED_STALL = 40 asks every reliable update to cut the FP64 |r|^2 to
    2^-40 of its best; at delta 0.1 each cuts it by about a hundred, so the first
    three reliable updates (a fall of about 1e-6) count as stalled and the solve
    finishes in FP64 CG from the accumulated solution: one restart, converged,
    and the oracle's bar.  The default (k = 1, halving) never falls back here.
    With x cycles of 3 and 4 (the default) the fallback may come inside a
    cycle, whose directions the accumulated solution must then take."""
    dims, lat, setup, b, ref = case
    lat.set_option(capi.QCD_OPT_MIXED_STALL, 40)
    lat.set_option(capi.QCD_OPT_X_CYCLE, cycle)
    try:
        x, st = lat.solve(to_dev(b), prec="mixed", tol=1e-12)
    finally:
        lat.set_option(capi.QCD_OPT_MIXED_STALL, 1)
        lat.set_option(capi.QCD_OPT_X_CYCLE, 4)
    print(f"  fallback: iters={st['iters']} ru={st['reliable_updates']} restarts={st['restarts']}", flush=True)
    assert st["restarts"] == 1 and st["converged"] == 1
    assert 3 <= st["reliable_updates"] <= 4
    assert rel_err(x, ref.x) < 1e-10 and st["true_rel_res"] < 1e-10
    x2, st2 = lat.solve(to_dev(b), prec="mixed", tol=1e-12)
    assert st2["restarts"] == 0 and st2["reliable_updates"] > 3
    for bad in (0, 61):
        with pytest.raises(QCDError, match="EINVAL"):
            lat.set_option(capi.QCD_OPT_MIXED_STALL, bad)


# ---------------------------------------------------------------- x cycles
@pytest.mark.parametrize("cycle", [1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_x_cycle_solve_parity(case, prec, cycle):
    """QCD_OPT_X_CYCLE = n keeps the search directions of n iterations and updates
    x once per n; the mixed solver's reliable updates (at least five here, so
    some fall inside a cycle for n > 1) fold the pending directions in.  Every
    n meets the oracle's bar (the default, 4, is the solve test above)."""
    dims, lat, setup, b, ref = case
    lat.set_option(capi.QCD_OPT_X_CYCLE, cycle)
    try:
        x, st = lat.solve(to_dev(b), prec=prec, tol=1e-12)
    finally:
        lat.set_option(capi.QCD_OPT_X_CYCLE, 4)
    print(f"  {prec} cycle={cycle}: iters={st['iters']} ru={st['reliable_updates']}", flush=True)
    assert st["converged"] == 1 and st["restarts"] == 0
    assert rel_err(x, ref.x) < 1e-10 and st["true_rel_res"] < 1e-10
    if prec == "mixed":
        assert st["reliable_updates"] >= 5


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_x_cycle_stopped_at_every_position(prec):
    """Capped at m = 1 .. 9 iterations, the recurrence stops at every position of
    cycles of 2, 3 and 4 iterations (the mixed solver, with two iterations in
    flight, runs m + 1 and folds the unfinished cycle in at its one reliable
    update).  The recurrence (r, p, alpha, beta) reads x only at a reliable
    update, and delta_reliable = 1e-6 allows none before the cap, so the iterate
    must equal that of cycle 1 (x updated every iteration) up to the rounding
    of the sums (FP64; FP32 for the mixed x_lo): a direction dropped or taken
    twice would move it by alpha_k p_k, which at these m is far larger (checked:
    consecutive m differ by much more than the bar)."""
    dims = (4, 4, 4, 4)
    lat, setup, u, ud = make_case(dims, 0.3, 0.12, 1.0, 0)
    b = to_dev(synth.gaussian_source(dims, 0, 0))
    bar = 1e-13 if prec == "fp64" else 1e-6
    prev = None
    try:
        for m in range(1, 10):
            xs = {}
            for cyc in (1, 2, 3, 4):
                lat.set_option(capi.QCD_OPT_X_CYCLE, cyc)
                xs[cyc], st = lat.solve(b, prec=prec, tol=1e-14, max_iter=m, delta_reliable=1e-6,
                                        raise_on_noconv=False)
                assert st["status"] == "QCD_ENOCONV"
                if prec == "fp64":
                    assert st["iters"] == m
                else:
                    assert st["reliable_updates"] == 1
            for cyc in (2, 3, 4):
                assert rel_err(xs[cyc], xs[1]) < bar, (m, cyc)
            if prev is not None:
                assert rel_err(xs[1], prev) > 1e3 * bar, m
            prev = xs[1]
    finally:
        lat.set_option(capi.QCD_OPT_X_CYCLE, 4)
        lat.close()


def test_x_cycle_rejects_out_of_range():
    lat = Lattice((4, 4, 4, 4), 0.12, 1.0)
    for bad in (0, 5, -1):
        with pytest.raises(QCDError, match="EINVAL"):
            lat.set_option(capi.QCD_OPT_X_CYCLE, bad)
    lat.close()
