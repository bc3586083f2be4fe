"""Python objects over the C-ABI: a lattice context, the solver, the force
as a ``torch.autograd.Function`` and one HMD step.

The computation is the hot path of the dynamical clover-fermion R-algorithm
application of arXiv:0910.0262 (abstract; section 1): the even-odd
preconditioned Wilson-clover operator, CG on Mhat^dag Mhat, and the fermion
force.  Tensors live in GPU memory (torch allocates them); every operation
is a call into libcloverqcd.
"""
from __future__ import annotations

import torch

from . import capi
from .capi import (QCD_FP64, QCD_MIXED, QCD_OP_M, QCD_OP_MDAG, QCD_OP_MHAT, QCD_OP_MHATDAG,  # noqa: F401
                   QCD_OP_MHATDAGMHAT, QCD_OPT_BLOCK, QCD_OPT_LINK_RECON, QCD_OPT_MIXED_CLOVER, QCDError)

_PREC = {"fp64": QCD_FP64, "mixed": QCD_MIXED, QCD_FP64: QCD_FP64, QCD_MIXED: QCD_MIXED}
_OPS = {"M": QCD_OP_M, "Mdag": QCD_OP_MDAG, "Mhat": QCD_OP_MHAT, "Mhatdag": QCD_OP_MHATDAG,
        "MdagM": QCD_OP_MHATDAGMHAT}


class Lattice:
    """One lattice on one GPU: gauge field, clover term and work buffers (owned by the library).

    dims = (Lx, Ly, Lz, Lt), all even.  Arrays use lexicographic site order
    (x fastest): gauge (Lt, Lz, Ly, Lx, 4, 3, 3) complex128, spinor
    (Lt, Lz, Ly, Lx, 4, 3) complex128, even-site vectors (V/2, 4, 3)."""

    def __init__(self, dims, kappa=0.125, csw=1.0, t_boundary=-1, device=0, stream=None):
        self.dims = tuple(int(d) for d in dims)
        lx, ly, lz, lt = self.dims
        self.V = lx * ly * lz * lt
        self.Vh = self.V // 2
        self.device = torch.device("cuda", device)
        self._ctx = capi.qcd_create(self.dims, device, stream)
        self.set_params(kappa, csw, t_boundary)

    # -- lifetime
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            capi.qcd_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ctx(self):
        return self._ctx

    # -- parameters and fields
    def set_params(self, kappa, csw, t_boundary=-1):
        capi.qcd_set_params(self._ctx, kappa, csw, t_boundary)
        self.kappa, self.csw, self.t_boundary = float(kappa), float(csw), int(t_boundary)

    def set_option(self, option, value):
        capi.qcd_set_option(self._ctx, option, value)

    def load_gauge(self, U: torch.Tensor, build_clover: bool = True):
        capi.qcd_load_gauge(self._ctx, U, self.V)
        if build_clover:
            capi.qcd_build_clover(self._ctx)

    def store_gauge(self) -> torch.Tensor:
        lx, ly, lz, lt = self.dims
        U = torch.empty((lt, lz, ly, lx, 4, 3, 3), dtype=torch.complex128, device=self.device)
        capi.qcd_store_gauge(self._ctx, U, self.V)
        return U

    def build_clover(self):
        capi.qcd_build_clover(self._ctx)

    def load_clover(self, A: torch.Tensor):
        capi.qcd_load_clover(self._ctx, A, self.V)

    def get_clover(self):
        """(A [V, 2, 36], A_oo^{-1} [V/2, 2, 36]) in the packed Hermitian-block layout."""
        A = torch.empty((self.V, 2, 36), dtype=torch.float64, device=self.device)
        Ai = torch.empty((self.Vh, 2, 36), dtype=torch.float64, device=self.device)
        capi.qcd_get_clover(self._ctx, A, Ai, self.V)
        return A, Ai

    # -- operators
    def apply(self, op, psi: torch.Tensor, prec="fp64") -> torch.Tensor:
        code = _OPS.get(op, op)
        n = self.V if code in (QCD_OP_M, QCD_OP_MDAG) else self.Vh
        out = torch.empty_like(psi)
        capi.qcd_apply(self._ctx, code, _PREC[prec], psi, out, n)
        return out

    def solve(self, b: torch.Tensor, prec="fp64", tol=1e-10, max_iter=20000, pipeline_depth=2, delta_reliable=0.1,
              raise_on_noconv=True):
        """x with M x = b on the full lattice; returns (x, stats dict)."""
        x = torch.empty_like(b)
        p = capi.make_params(_PREC[prec], tol, max_iter, pipeline_depth, delta_reliable)
        rc, st = capi.qcd_solve(self._ctx, p, b, x, self.V, raise_on_noconv)
        st["status"] = capi.STATUS_NAMES[rc]
        return x, st

    def solve_multi(self, b: torch.Tensor, prec="fp64", tol=1e-10, max_iter=20000, pipeline_depth=2,
                    delta_reliable=0.1, raise_on_noconv=True):
        """Solve M x_k = b_k for b of shape (n, Lt, Lz, Ly, Lx, 4, 3), n <= 16, in one interleaved
        multi-source solve; returns (x, [stats dict] * n)."""
        x = torch.empty_like(b)
        p = capi.make_params(_PREC[prec], tol, max_iter, pipeline_depth, delta_reliable)
        rc, sts = capi.qcd_solve_multi(self._ctx, p, b, x, self.V, raise_on_noconv)
        for st in sts:
            st["status"] = capi.STATUS_NAMES[rc]
        return x, sts

    def action_force(self, phi: torch.Tensor, prec="fp64", tol=1e-12, max_iter=20000, pipeline_depth=2,
                     delta_reliable=0.1, want_F=True, want_X=True):
        """S = phi^dag (Mhat^dag Mhat)^{-1} phi and its derivatives.

        Returns (S, G, F, X, stats): G = dS/dRe U + i dS/dIm U, shape of the gauge
        field; F the su(3) force coefficients (..., 4, 8); X the solution."""
        lx, ly, lz, lt = self.dims
        G = torch.empty((lt, lz, ly, lx, 4, 3, 3), dtype=torch.complex128, device=self.device)
        F = torch.empty((lt, lz, ly, lx, 4, 8), dtype=torch.float64, device=self.device) if want_F else None
        X = torch.empty((self.Vh, 4, 3), dtype=torch.complex128, device=self.device) if want_X else None
        p = capi.make_params(_PREC[prec], tol, max_iter, pipeline_depth, delta_reliable)
        S, st = capi.qcd_action_force(self._ctx, p, phi, G, F, X, self.V)
        return S, G, F, X, st

    def hmd_step(self, U: torch.Tensor, P: torch.Tensor, xi: torch.Tensor, dt: float, prec="fp64", tol=1e-12,
                 max_iter=20000, pipeline_depth=2, delta_reliable=0.1):
        """One HMD step in place on U and P; returns (S at the midpoint, stats)."""
        p = capi.make_params(_PREC[prec], tol, max_iter, pipeline_depth, delta_reliable)
        return capi.qcd_hmd_step(self._ctx, dt, U, P, xi, p, self.V)

    def gauge_action_force(self, beta: float, want_G=True, want_F=True):
        """Wilson plaquette action S_g and its derivative (G, F) on the loaded gauge field."""
        G, F = self._force_buffers(want_G, want_F)
        S = capi.qcd_gauge_action_force(self._ctx, beta, G, F, self.V)
        return S, G, F

    def clover_det_action_force(self, want_G=True, want_F=True):
        """S_det = -2 sum_odd ln det A and its derivative (G, F)."""
        G, F = self._force_buffers(want_G, want_F)
        S = capi.qcd_clover_det_action_force(self._ctx, G, F, self.V)
        return S, G, F

    def md_trajectory(self, U: torch.Tensor, P: torch.Tensor, xi: torch.Tensor | None, dt: float, n_steps: int,
                      beta: float = 0.0, n_f: float = 2.0, clover_det: bool = True, reunitarize: bool = False,
                      prec="fp64", tol=1e-12, max_iter=20000, pipeline_depth=2, delta_reliable=0.1,
                      raise_on_noconv=True):
        """One R-algorithm trajectory in place on U and P; xi is (n_steps, V/2, 4, 3).

        Returns (actions, stats): actions[k] = (S_f, S_g, S_det) at step k's force evaluation."""
        md = capi.make_md_params(dt, n_steps, beta, n_f, clover_det, reunitarize)
        p = capi.make_params(_PREC[prec], tol, max_iter, pipeline_depth, delta_reliable) if n_f != 0 else None
        rc, acts, st = capi.qcd_md_trajectory(self._ctx, md, U, P, xi, p, self.V, raise_on_noconv)
        st["status"] = capi.STATUS_NAMES[rc]
        return acts, st

    def _force_buffers(self, want_G, want_F):
        lx, ly, lz, lt = self.dims
        G = torch.empty((lt, lz, ly, lx, 4, 3, 3), dtype=torch.complex128, device=self.device) if want_G else None
        F = torch.empty((lt, lz, ly, lx, 4, 8), dtype=torch.float64, device=self.device) if want_F else None
        return G, F

    def encode_half(self, psi: torch.Tensor):
        n = psi.numel() // 12
        codes = torch.empty((n, 24), dtype=torch.float16, device=self.device)
        scale = torch.empty((n,), dtype=torch.float32, device=self.device)
        capi.qcd_encode_half(self._ctx, psi, codes, scale)
        return codes, scale

    def time_stencil(self, prec="fp64", n=20):
        """(k1 ms/launch, k2 ms/launch, Mhat^dag Mhat ms/application) on the current fields."""
        return capi.qcd_time_stencil(self._ctx, _PREC[prec], n)

    def time_stencil_multi(self, n_rhs, prec="mixed", n=20):
        """(k1, k2, Mhat^dag Mhat) ms per launch / application for n_rhs interleaved right-hand sides."""
        return capi.qcd_time_stencil_multi(self._ctx, _PREC[prec], n_rhs, n)

    def stream_copy(self, dst: torch.Tensor, src: torch.Tensor):
        capi.qcd_stream_copy(self._ctx, dst, src)


class CloverForce(torch.autograd.Function):
    """S(U, phi) = phi^dag (Mhat^dag Mhat)^{-1} phi with a hand-written adjoint.

    forward runs the solve and the force kernels of the library; backward
    returns grad_U = gS * G (G = dS/dRe U + i dS/dIm U, the PyTorch convention
    for a real function of complex inputs) and grad_phi = 2 gS X."""

    @staticmethod
    def forward(ctx, U, phi, lattice: Lattice, prec="fp64", tol=1e-12):
        lattice.load_gauge(U.detach().contiguous())
        S, G, _, X, st = lattice.action_force(phi.detach().contiguous(), prec=prec, tol=tol, want_F=False)
        ctx.save_for_backward(G, X)
        ctx.stats = st
        return torch.tensor(S, dtype=torch.float64, device=U.device)

    @staticmethod
    def backward(ctx, gS):
        G, X = ctx.saved_tensors
        return gS * G, 2.0 * gS * X, None, None, None
