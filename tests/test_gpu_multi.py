"""GPU parity of the multi-source solve (right-hand sides interleaved site by
site, links and clover read once per site for all of them) against the oracle.

Bar: as for single solves, relative solution error <= 1e-10 per right-hand
side against the oracle's FP64 solution, both to tol 1e-12, and the oracle's
operator applied to each GPU solution leaves a relative residual <= 1e-10.
At 32^3 x 64 (the benchmark's lattice and launch configuration) and 24^3 x 48
the oracle does not solve (hours per source); there the oracle's operator M is
applied to GPU solutions (seconds each) and the relative residual must be
<= 5e-10."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_0910_0262_amd import Lattice, QCDError, capi, synth

from ._gpu_helpers import make_case, rel_err, to_dev

pytestmark = pytest.mark.gpu

CASES = [
    ((4, 4, 4, 4), 0.3, 0.12, 1.0, 0),
    ((6, 4, 2, 6), 0.5, 0.124, 1.3, 1),
    ((8, 8, 16, 16), 0.5, 0.124, 1.0, 2),
]
IDS = ["4^4", "6x4x2x6", "8x8x16x16"]


@pytest.fixture(scope="module", params=CASES, ids=IDS)
def case(request):
    dims, w, k, c, seed = request.param
    print(f"[multi case dims={dims} width={w} kappa={k} seed={seed}]", flush=True)
    lat, setup, u, ud = make_case(dims, w, k, c, seed)
    bs = np.stack([synth.gaussian_source(dims, seed, j) for j in range(5)])
    refs = [O.solve_full(setup, torch.as_tensor(b), 1e-13).x for b in bs]
    yield dims, lat, setup, bs, refs
    lat.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [1, 3, 4, 5])
def test_multi_solve_parity(case, prec, n):
    dims, lat, setup, bs, refs = case
    x, sts = lat.solve_multi(to_dev(bs[:n]), prec=prec, tol=1e-12)
    print(f"  {prec} n={n}: iters={sts[0]['iters']} ru={sts[0]['reliable_updates']}", flush=True)
    assert x.shape == (n,) + bs.shape[1:]
    for j in range(n):
        assert sts[j]["converged"] == 1
        assert sts[j]["true_rel_res"] < 1e-10
        if prec == "mixed":
            assert sts[j]["reliable_updates"] >= 5
        assert rel_err(x[j], refs[j]) < 1e-10, j
        r = torch.as_tensor(bs[j]) - setup.M(x[j].cpu())
        assert float(torch.linalg.norm(r) / torch.linalg.norm(torch.as_tensor(bs[j]))) < 1e-10


@pytest.mark.parametrize("cycle", [1, 3])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_multi_x_cycles(case, prec, cycle):
    """Five right-hand sides converge at different iterations, so with x cycles
    of 3 (and 4, the default, in the solve test above) each FP64 recurrence
    stops at its own position in the cycle and takes its pending directions
    there; every solution meets the oracle's bar."""
    dims, lat, setup, bs, refs = case
    lat.set_option(capi.QCD_OPT_X_CYCLE, cycle)
    try:
        x, sts = lat.solve_multi(to_dev(bs), prec=prec, tol=1e-12)
    finally:
        lat.set_option(capi.QCD_OPT_X_CYCLE, 4)
    print(f"  {prec} cycle={cycle}: iters={[s['iters'] for s in sts]}", flush=True)
    for j in range(len(bs)):
        assert sts[j]["converged"] == 1 and sts[j]["true_rel_res"] < 1e-10
        assert rel_err(x[j], refs[j]) < 1e-10, j


def test_multi_matches_single_and_is_deterministic(case):
    dims, lat, setup, bs, refs = case
    b = to_dev(bs[:4])
    xm1, s1 = lat.solve_multi(b, prec="fp64", tol=1e-10)
    xm2, s2 = lat.solve_multi(b, prec="fp64", tol=1e-10)
    assert torch.equal(xm1, xm2)
    for j in range(4):
        xs, _ = lat.solve(b[j].contiguous(), prec="fp64", tol=1e-10)
        assert rel_err(xm1[j], xs) < 1e-8
    ym1, _ = lat.solve_multi(b, prec="mixed", tol=1e-10)
    ym2, _ = lat.solve_multi(b, prec="mixed", tol=1e-10)
    assert torch.equal(ym1, ym2)


def test_mixed_multi_matches_single_source_mixed(case):
    """The multi-source mixed kernels read all nine binary16 link entries, the
    single-source ones two rows and rebuild the third: both solutions meet the
    FP64 residual, so they agree to within cond * tol."""
    dims, lat, setup, bs, refs = case
    b = to_dev(bs[:3])
    xm, sm = lat.solve_multi(b, prec="mixed", tol=1e-12)
    for j in range(3):
        xs, ss = lat.solve(b[j].contiguous(), prec="mixed", tol=1e-12)
        assert rel_err(xm[j], xs) < 1e-9, j
        assert sm[j]["true_rel_res"] < 1e-10 and ss["true_rel_res"] < 1e-10


def test_multi_with_fp32_clover(case):
    """The multi-source mixed kernels with the FP32 clover storage option."""
    dims, lat, setup, bs, refs = case
    lat.set_option(capi.QCD_OPT_MIXED_CLOVER, 32)
    try:
        x, sts = lat.solve_multi(to_dev(bs[:3]), prec="mixed", tol=1e-12)
    finally:
        lat.set_option(capi.QCD_OPT_MIXED_CLOVER, 16)
    for j in range(3):
        assert sts[j]["converged"] == 1
        assert rel_err(x[j], refs[j]) < 1e-10, j


@pytest.mark.parametrize("block", [64, 128, 256])
def test_workgroup_sizes(case, block):
    """Multi-source solves default to 256-thread workgroups and single-source
    ones to 64; every allowed size gives the oracle's solutions (and, with
    fewer partial sums per right-hand side, a different but fixed summation
    order, so each size is deterministic)."""
    dims, lat, setup, bs, refs = case
    b = to_dev(bs[:4])
    lat.set_option(capi.QCD_OPT_BLOCK, block)
    try:
        for prec in ("fp64", "mixed"):
            x, sts = lat.solve_multi(b, prec=prec, tol=1e-12)
            x2, _ = lat.solve_multi(b, prec=prec, tol=1e-12)
            assert torch.equal(x, x2), prec
            for j in range(4):
                assert sts[j]["converged"] == 1
                assert rel_err(x[j], refs[j]) < 1e-10, (prec, j)
            x1, st1 = lat.solve(b[0].contiguous(), prec=prec, tol=1e-12)
            assert st1["converged"] == 1
            assert rel_err(x1, refs[0]) < 1e-10, prec
    finally:
        lat.set_option(capi.QCD_OPT_BLOCK, 0)


def test_links_rederived_after_gauge_reload():
    """A second gauge field loaded into the same context reaches every link
    copy the multi-source kernels read."""
    dims, kappa, csw = (4, 4, 4, 8), 0.125, 1.0
    lat, setup, u, ud = make_case(dims, 0.3, kappa, csw, 8)
    bs = np.stack([synth.gaussian_source(dims, 8, j) for j in range(2)])
    lat.solve_multi(to_dev(bs), prec="mixed", tol=1e-10)
    u2 = synth.random_su3_field(dims, 0.4, 9)
    lat.load_gauge(to_dev(u2))
    setup2 = O.CloverSetup(torch.as_tensor(u2), kappa, csw)
    x, sts = lat.solve_multi(to_dev(bs), prec="mixed", tol=1e-12)
    for j in range(2):
        ref = O.solve_full(setup2, torch.as_tensor(bs[j]), 1e-13).x
        assert rel_err(x[j], ref) < 1e-10, j
    lat.close()


def test_zero_and_scaled_sources():
    """A zero source among others gives x = 0; sources of very different norms
    each meet the relative tolerance."""
    dims, kappa, csw = (4, 4, 4, 8), 0.125, 1.0
    lat, setup, u, ud = make_case(dims, 0.3, kappa, csw, 4)
    bs = np.stack([synth.gaussian_source(dims, 4, j) for j in range(3)])
    bs[1] = 0.0
    bs[2] *= 1e6
    for prec in ("fp64", "mixed"):
        x, sts = lat.solve_multi(to_dev(bs), prec=prec, tol=1e-12)
        assert float(torch.abs(x[1]).max()) == 0.0
        for j in (0, 2):
            ref = O.solve_full(setup, torch.as_tensor(bs[j]), 1e-13).x
            assert rel_err(x[j], ref) < 1e-10, (prec, j)
            assert sts[j]["converged"] == 1
        assert sts[1]["converged"] == 1
    lat.close()


def test_sixteen_sources_and_limits():
    dims = (4, 4, 4, 4)
    lat, setup, u, ud = make_case(dims, 0.3, 0.12, 1.0, 5)
    bs = np.stack([synth.gaussian_source(dims, 5, j) for j in range(16)])
    x, sts = lat.solve_multi(to_dev(bs), prec="mixed", tol=1e-12)
    for j in (0, 7, 15):
        ref = O.solve_full(setup, torch.as_tensor(bs[j]), 1e-13).x
        assert rel_err(x[j], ref) < 1e-10
    assert all(s["converged"] == 1 for s in sts)
    with pytest.raises(ValueError):
        lat.solve_multi(to_dev(np.concatenate([bs, bs[:1]])))
    # a 16-source set then a 2-source call reuses the larger buffers
    x2, _ = lat.solve_multi(to_dev(bs[:2]), prec="fp64", tol=1e-12)
    assert rel_err(x2[1], O.solve_full(setup, torch.as_tensor(bs[1]), 1e-13).x) < 1e-10
    lat.close()


def test_max_iter_reports_noconv_for_all():
    dims = (4, 4, 4, 4)
    lat, setup, u, ud = make_case(dims, 0.3, 0.12, 1.0, 6)
    bs = np.stack([synth.gaussian_source(dims, 6, j) for j in range(2)])
    with pytest.raises(QCDError, match="ENOCONV"):
        lat.solve_multi(to_dev(bs), prec="fp64", tol=1e-12, max_iter=3)
    x, sts = lat.solve_multi(to_dev(bs), prec="fp64", tol=1e-12, max_iter=3, raise_on_noconv=False)
    assert all(s["converged"] == 0 for s in sts)
    assert torch.isfinite(x).all()
    lat.close()


def test_context_state_after_multi_solve():
    """Single-source calls and the force work as before after a multi-source solve."""
    dims, kappa, csw = (4, 4, 4, 4), 0.12, 1.0
    lat, setup, u, ud = make_case(dims, 0.3, kappa, csw, 7)
    b = synth.gaussian_source(dims, 7, 0)
    x0, _ = lat.solve(to_dev(b), prec="fp64", tol=1e-12)
    lat.solve_multi(to_dev(np.stack([b, b, b])), prec="mixed", tol=1e-10)
    x1, _ = lat.solve(to_dev(b), prec="fp64", tol=1e-12)
    assert torch.equal(x0, x1)
    phi = setup.Mhat_dag(torch.as_tensor(synth.heatbath_xi(dims, 7)))
    S, G, X, _ = O.action_and_gradient(torch.as_tensor(u), kappa, csw, phi, tol=1e-14)
    S_g, G_g, _, _, _ = lat.action_force(to_dev(phi), tol=1e-12)
    assert abs(S_g - S) < 1e-10 * abs(S)
    lat.close()


@pytest.fixture(scope="module")
def oracle_32():
    """The oracle's operator on the benchmark's lattice: 32^3 x 64, kappa 0.1255,
    c_sw 1, links of width 0.2 from seed 0 (its clover setup takes ~10 s)."""
    dims, kappa, csw = (32, 32, 32, 64), 0.1255, 1.0
    print("[oracle setup 32^3x64]", flush=True)
    u = synth.random_su3_field(dims, 0.2, 0)
    return u, O.CloverSetup(torch.as_tensor(u), kappa, csw)


def _oracle_residual(setup, b, x):
    """|b - M x| / |b| with the oracle's full-lattice FP64 operator."""
    bc = b.cpu()
    return float(torch.linalg.norm(bc - setup.M(x.cpu())) / torch.linalg.norm(bc))


@pytest.mark.parametrize("block", [0, 64])
def test_full_lattice_eight_sources(block, oracle_32):
    """32^3 x 64, 8 sources, tol 1e-10, as timed by the benchmark.  The oracle's
    FP64 operator M applied to sources 0 and 5 of each precision leaves a
    relative residual <= 5e-10 (the stopping test is on the normal equations;
    single solves land at 1-2e-10); sources 3 and 7 are checked the same way
    with the library's FP64 operator, and source 5 agrees with its
    single-source solve to within cond * tol.  The default workgroups leave
    32768 partial sums per right-hand side, 64-thread ones 131072: both are
    folded in spans before the finalisation kernels."""
    u, setup = oracle_32
    dims, kappa, csw = (32, 32, 32, 64), 0.1255, 1.0
    print(f"[multi 32^3x64, 8 sources, block {block}]", flush=True)
    lat = Lattice(dims, kappa, csw)
    lat.set_option(capi.QCD_OPT_BLOCK, block)
    lat.load_gauge(to_dev(u))
    b = torch.stack([to_dev(synth.gaussian_source(dims, 0, k)) for k in range(8)])
    for prec in ("mixed", "fp64"):
        x, sts = lat.solve_multi(b, prec=prec, tol=1e-10)
        print(f"  {prec}: iters={sts[0]['iters']} ru={sts[0]['reliable_updates']} "
              f"seconds={sts[0]['seconds']:.3f}", flush=True)
        for k in range(8):
            assert sts[k]["converged"] == 1
        for k in (0, 5):
            res = _oracle_residual(setup, b[k], x[k])
            print(f"    source {k}: oracle residual {res:.3e}", flush=True)
            assert res < 5e-10, (prec, k, res)
        for k in (3, 7):
            r = b[k] - lat.apply("M", x[k].contiguous())
            assert float(torch.linalg.norm(r) / torch.linalg.norm(b[k])) < 5e-10, (prec, k)
        xs, _ = lat.solve(b[5].contiguous(), prec=prec, tol=1e-10)
        assert rel_err(x[5], xs) < 1e-7
        del x
    lat.close()


def test_ragged_partial_fold():
    """24^3 x 48 with 8 sources and 64-thread workgroups leaves 41472 partial
    sums per right-hand side: ten full spans of 4096 and a last one of 512 are
    folded before the finalisation kernels.  The oracle's FP64 operator on
    sources 0 and 4, and the library's on source 7, leave a relative residual
    <= 5e-10, and each solution matches the solve at the default workgroup
    size (which does not fold at this size)."""
    dims, kappa, csw = (24, 24, 24, 48), 0.1255, 1.0
    vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
    assert vh * 8 // 64 == 41472 and 41472 % 4096 == 512
    print("[multi 24^3x48, 8 sources, ragged fold: oracle setup]", flush=True)
    u = synth.random_su3_field(dims, 0.2, 3)
    setup = O.CloverSetup(torch.as_tensor(u), kappa, csw)
    lat = Lattice(dims, kappa, csw)
    lat.load_gauge(to_dev(u))
    b = torch.stack([to_dev(synth.gaussian_source(dims, 3, k)) for k in range(8)])
    try:
        for prec in ("mixed", "fp64"):
            lat.set_option(capi.QCD_OPT_BLOCK, 64)
            x, sts = lat.solve_multi(b, prec=prec, tol=1e-10)
            lat.set_option(capi.QCD_OPT_BLOCK, 0)
            xd, _ = lat.solve_multi(b, prec=prec, tol=1e-10)
            print(f"  {prec}: iters={sts[0]['iters']}", flush=True)
            for k in (0, 4, 7):
                assert sts[k]["converged"] == 1
                if k == 7:
                    r = b[k] - lat.apply("M", x[k].contiguous())
                    res = float(torch.linalg.norm(r) / torch.linalg.norm(b[k]))
                else:
                    res = _oracle_residual(setup, b[k], x[k])
                assert res < 5e-10, (prec, k, res)
                assert rel_err(x[k], xd[k]) < 1e-7, (prec, k)
            del x, xd
    finally:
        lat.set_option(capi.QCD_OPT_BLOCK, 0)
        lat.close()
