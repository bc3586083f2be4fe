"""ctypes binding of libcloverqcd (include/cloverqcd.h), one Python function per C entry point.

Argument marshalling only: every function checks dtype / shape / device of
the torch tensors it is handed, passes their data pointers and sizes to the
C library, and raises :class:`QCDError` on a non-OK status.  All arithmetic
happens in the library's HIP kernels; there is no fallback path.  If the
shared library is missing it is built from the package sources (hipcc); if
it cannot be loaded, importing a function raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcloverqcd.so")

QCD_OK, QCD_EINVAL, QCD_ESTATE, QCD_ENOMEM, QCD_EHIP, QCD_ENOCONV, QCD_ENAN, QCD_ECLOVER = 0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "QCD_OK", -1: "QCD_EINVAL", -2: "QCD_ESTATE", -3: "QCD_ENOMEM", -4: "QCD_EHIP",
                -5: "QCD_ENOCONV", -6: "QCD_ENAN", -7: "QCD_ECLOVER"}
QCD_FP64, QCD_MIXED = 0, 1
QCD_OP_M, QCD_OP_MDAG, QCD_OP_MHAT, QCD_OP_MHATDAG, QCD_OP_MHATDAGMHAT = 0, 1, 2, 3, 4
QCD_OPT_LINK_RECON, QCD_OPT_MIXED_CLOVER, QCD_OPT_BLOCK, QCD_OPT_GRAPH, QCD_OPT_SMALL_GRID = 0, 1, 2, 3, 4
QCD_OPT_MIXED_STALL, QCD_OPT_COMPACT_CLOVER, QCD_OPT_X_CYCLE = 5, 6, 7


class QCDError(RuntimeError):
    def __init__(self, code: int, message: str):
        self.code = code
        self.status = STATUS_NAMES.get(code, str(code))
        super().__init__(f"{self.status}: {message}")


class SolverParams(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int), ("max_iter", ctypes.c_int), ("pipeline_depth", ctypes.c_int),
                ("tol", ctypes.c_double), ("delta_reliable", ctypes.c_double)]


class SolverStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("converged", ctypes.c_int),
                ("restarts", ctypes.c_int), ("normal_rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("seconds", ctypes.c_double), ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class MDParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("beta", ctypes.c_double), ("n_f", ctypes.c_double),
                ("n_steps", ctypes.c_int), ("clover_det", ctypes.c_int), ("reunitarize", ctypes.c_int)]


_lock = threading.Lock()
_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
SIGNATURES = {
    "qcd_version": ([], _I),
    "qcd_last_error": ([], ctypes.c_char_p),
    "qcd_create": ([ctypes.POINTER(ctypes.c_int), _I, ctypes.c_size_t, ctypes.POINTER(_P)], _I),
    "qcd_destroy": ([_P], _I),
    "qcd_set_params": ([_P, _D, _D, _I], _I),
    "qcd_set_option": ([_P, _I, _I], _I),
    "qcd_load_gauge": ([_P, _P], _I),
    "qcd_store_gauge": ([_P, _P], _I),
    "qcd_build_clover": ([_P], _I),
    "qcd_load_clover": ([_P, _P], _I),
    "qcd_get_clover": ([_P, _P, _P], _I),
    "qcd_apply": ([_P, _I, _I, _P, _P], _I),
    "qcd_solve": ([_P, ctypes.POINTER(SolverParams), _P, _P, ctypes.POINTER(SolverStats)], _I),
    "qcd_solve_multi": ([_P, ctypes.POINTER(SolverParams), _I, _P, _P, ctypes.POINTER(SolverStats)], _I),
    "qcd_action_force": ([_P, ctypes.POINTER(SolverParams), _P, ctypes.POINTER(_D), _P, _P, _P,
                          ctypes.POINTER(SolverStats)], _I),
    "qcd_hmd_step": ([_P, _D, _P, _P, _P, ctypes.POINTER(SolverParams), ctypes.POINTER(_D),
                      ctypes.POINTER(SolverStats)], _I),
    "qcd_gauge_action_force": ([_P, _D, ctypes.POINTER(_D), _P, _P], _I),
    "qcd_gauge_force_noalloc": ([_P, _D, _P, _P], _I),
    "qcd_clover_det_action_force": ([_P, ctypes.POINTER(_D), _P, _P], _I),
    "qcd_md_trajectory": ([_P, ctypes.POINTER(MDParams), _P, _P, _P, ctypes.POINTER(SolverParams),
                           ctypes.POINTER(_D), ctypes.POINTER(SolverStats)], _I),
    "qcd_encode_half": ([_P, _I, _P, _P, _P], _I),
    "qcd_time_stencil": ([_P, _I, _I, ctypes.POINTER(ctypes.c_double)], _I),
    "qcd_time_stencil_multi": ([_P, _I, _I, _I, ctypes.POINTER(ctypes.c_double)], _I),
    "qcd_stream_copy": ([_P, _P, _P, ctypes.c_uint64], _I),
}


def lib() -> ctypes.CDLL:
    """Load libcloverqcd.so (building it first if it is not there)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            from .csrc.build import build

            build()
        handle = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = res
        _lib = handle
        return _lib


def last_error() -> str:
    return lib().qcd_last_error().decode()


def check(rc: int) -> int:
    if rc != QCD_OK:
        raise QCDError(rc, last_error())
    return rc


def _ptr(t, dtype, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be in GPU memory")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------- one function per entry point
def qcd_version() -> int:
    return lib().qcd_version()


def qcd_create(dims, device: int = 0, stream: int | None = None) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream(device).cuda_stream
    d = (ctypes.c_int * 4)(*[int(v) for v in dims])
    out = ctypes.c_void_p()
    check(lib().qcd_create(d, int(device), ctypes.c_size_t(int(stream)), ctypes.byref(out)))
    return out


def qcd_destroy(ctx) -> None:
    check(lib().qcd_destroy(ctx))


def qcd_set_params(ctx, kappa: float, csw: float, t_boundary: int = -1) -> None:
    check(lib().qcd_set_params(ctx, float(kappa), float(csw), int(t_boundary)))


def qcd_set_option(ctx, option: int, value: int) -> None:
    check(lib().qcd_set_option(ctx, int(option), int(value)))


def qcd_load_gauge(ctx, U: torch.Tensor, volume: int) -> None:
    check(lib().qcd_load_gauge(ctx, _ptr(U, torch.complex128, volume * 36, "U")))


def qcd_store_gauge(ctx, U: torch.Tensor, volume: int) -> None:
    check(lib().qcd_store_gauge(ctx, _ptr(U, torch.complex128, volume * 36, "U")))


def qcd_build_clover(ctx) -> None:
    check(lib().qcd_build_clover(ctx))


def qcd_load_clover(ctx, A: torch.Tensor, volume: int) -> None:
    check(lib().qcd_load_clover(ctx, _ptr(A, torch.float64, volume * 72, "A")))


def qcd_get_clover(ctx, A: torch.Tensor | None, Ainv: torch.Tensor | None, volume: int) -> None:
    check(lib().qcd_get_clover(ctx, _ptr(A, torch.float64, volume * 72, "A"),
                               _ptr(Ainv, torch.float64, volume * 36, "Ainv")))


def qcd_apply(ctx, op: int, prec: int, src: torch.Tensor, dst: torch.Tensor, n_sites: int) -> None:
    check(lib().qcd_apply(ctx, int(op), int(prec), _ptr(src, torch.complex128, n_sites * 12, "in"),
                          _ptr(dst, torch.complex128, n_sites * 12, "out")))


def make_params(prec=QCD_FP64, tol=1e-10, max_iter=20000, pipeline_depth=2, delta_reliable=0.1) -> SolverParams:
    return SolverParams(int(prec), int(max_iter), int(pipeline_depth), float(tol), float(delta_reliable))


def qcd_solve(ctx, params: SolverParams, b: torch.Tensor, x: torch.Tensor, volume: int,
              raise_on_noconv: bool = True) -> tuple[int, dict]:
    st = SolverStats()
    rc = lib().qcd_solve(ctx, ctypes.byref(params), _ptr(b, torch.complex128, volume * 12, "b"),
                         _ptr(x, torch.complex128, volume * 12, "x"), ctypes.byref(st))
    if rc != QCD_OK and (raise_on_noconv or rc != QCD_ENOCONV):
        check(rc)
    return rc, st.as_dict()


QCD_MAX_RHS = 16


def qcd_solve_multi(ctx, params: SolverParams, b: torch.Tensor, x: torch.Tensor, volume: int,
                    raise_on_noconv: bool = True) -> tuple[int, list]:
    """b, x: complex128 (n, ..., V sites, 4, 3) with n <= 16 right-hand sides; returns (status, [stats] * n)."""
    n = b.shape[0]
    if not 1 <= n <= QCD_MAX_RHS:
        raise ValueError(f"1 <= n_rhs <= {QCD_MAX_RHS} required, got {n}")
    st = (SolverStats * n)()
    rc = lib().qcd_solve_multi(ctx, ctypes.byref(params), n, _ptr(b, torch.complex128, n * volume * 12, "b"),
                               _ptr(x, torch.complex128, n * volume * 12, "x"), st)
    if rc != QCD_OK and (raise_on_noconv or rc != QCD_ENOCONV):
        check(rc)
    return rc, [st[k].as_dict() for k in range(n)]


def qcd_action_force(ctx, params: SolverParams, phi: torch.Tensor, G: torch.Tensor, F: torch.Tensor | None,
                     X: torch.Tensor | None, volume: int) -> tuple[float, dict]:
    st = SolverStats()
    s = ctypes.c_double(0.0)
    vh = volume // 2
    check(lib().qcd_action_force(ctx, ctypes.byref(params), _ptr(phi, torch.complex128, vh * 12, "phi"),
                                 ctypes.byref(s), _ptr(G, torch.complex128, volume * 36, "G"),
                                 _ptr(F, torch.float64, volume * 32, "F"), _ptr(X, torch.complex128, vh * 12, "X"),
                                 ctypes.byref(st)))
    return s.value, st.as_dict()


def qcd_hmd_step(ctx, dt: float, U: torch.Tensor, P: torch.Tensor, xi: torch.Tensor, params: SolverParams,
                 volume: int) -> tuple[float, dict]:
    st = SolverStats()
    s = ctypes.c_double(0.0)
    check(lib().qcd_hmd_step(ctx, float(dt), _ptr(U, torch.complex128, volume * 36, "U"),
                             _ptr(P, torch.float64, volume * 32, "P"),
                             _ptr(xi, torch.complex128, volume // 2 * 12, "xi"), ctypes.byref(params),
                             ctypes.byref(s), ctypes.byref(st)))
    return s.value, st.as_dict()


def qcd_gauge_action_force(ctx, beta: float, G: torch.Tensor | None, F: torch.Tensor | None,
                           volume: int) -> float:
    s = ctypes.c_double(0.0)
    check(lib().qcd_gauge_action_force(ctx, float(beta), ctypes.byref(s),
                                       _ptr(G, torch.complex128, volume * 36, "G"),
                                       _ptr(F, torch.float64, volume * 32, "F")))
    return s.value


def qcd_gauge_force_noalloc(ctx, beta: float, G: torch.Tensor | None, F: torch.Tensor | None, volume: int) -> None:
    """Stream-ordered: the caller synchronises before reading G and F."""
    check(lib().qcd_gauge_force_noalloc(ctx, float(beta), _ptr(G, torch.complex128, volume * 36, "G"),
                                        _ptr(F, torch.float64, volume * 32, "F")))


def qcd_clover_det_action_force(ctx, G: torch.Tensor | None, F: torch.Tensor | None, volume: int) -> float:
    s = ctypes.c_double(0.0)
    check(lib().qcd_clover_det_action_force(ctx, ctypes.byref(s), _ptr(G, torch.complex128, volume * 36, "G"),
                                            _ptr(F, torch.float64, volume * 32, "F")))
    return s.value


def make_md_params(dt: float, n_steps: int, beta: float = 0.0, n_f: float = 2.0, clover_det: bool = True,
                   reunitarize: bool = False) -> MDParams:
    return MDParams(float(dt), float(beta), float(n_f), int(n_steps), int(bool(clover_det)), int(bool(reunitarize)))


def qcd_md_trajectory(ctx, md: MDParams, U: torch.Tensor, P: torch.Tensor, xi: torch.Tensor | None,
                      params: SolverParams | None, volume: int, raise_on_noconv: bool = True):
    """Returns (status, actions [n_steps][3] as a list of tuples, stats dict)."""
    st = SolverStats()
    acts = (ctypes.c_double * (3 * md.n_steps))()
    rc = lib().qcd_md_trajectory(ctx, ctypes.byref(md), _ptr(U, torch.complex128, volume * 36, "U"),
                                 _ptr(P, torch.float64, volume * 32, "P"),
                                 _ptr(xi, torch.complex128, md.n_steps * (volume // 2) * 12, "xi"),
                                 ctypes.byref(params) if params is not None else None, acts, ctypes.byref(st))
    if rc != QCD_OK and (raise_on_noconv or rc != QCD_ENOCONV):
        check(rc)
    out = [(acts[3 * k], acts[3 * k + 1], acts[3 * k + 2]) for k in range(md.n_steps)]
    return rc, out, st.as_dict()


def qcd_encode_half(ctx, src: torch.Tensor, codes: torch.Tensor, scale: torch.Tensor) -> None:
    n = src.numel() // 12
    check(lib().qcd_encode_half(ctx, n, _ptr(src, torch.complex128, n * 12, "in"),
                                _ptr(codes, torch.float16, n * 24, "codes"), _ptr(scale, torch.float32, n, "scale")))


def qcd_time_stencil(ctx, prec: int, n: int) -> tuple[float, float, float]:
    """(k1 ms per launch, k2 ms per launch, Mhat^dag Mhat ms per application)."""
    ms = (ctypes.c_double * 3)()
    check(lib().qcd_time_stencil(ctx, int(prec), int(n), ms))
    return ms[0], ms[1], ms[2]


def qcd_time_stencil_multi(ctx, prec: int, n_rhs: int, n: int) -> tuple[float, float, float]:
    """As qcd_time_stencil, each launch covering n_rhs interleaved right-hand sides."""
    ms = (ctypes.c_double * 3)()
    check(lib().qcd_time_stencil_multi(ctx, int(prec), int(n_rhs), int(n), ms))
    return ms[0], ms[1], ms[2]


def qcd_stream_copy(ctx, dst: torch.Tensor, src: torch.Tensor) -> None:
    if not (dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("stream copy needs contiguous GPU tensors")
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise ValueError("destination smaller than source")
    check(lib().qcd_stream_copy(ctx, ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                                ctypes.c_uint64(n)))
