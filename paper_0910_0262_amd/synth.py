"""Seeded synthetic inputs: gauge fields, sources, momenta, heat-bath noise.

This module holds no arithmetic of the method itself (no Dirac operator, no
clover term, no solver, no force).  It only draws the random inputs that both
the CPU oracle and the GPU library consume, so the two see bit-identical
arrays.  Every array is a NumPy complex128 / float64 array in host memory, in
the site order used throughout the project:

    site index i = x + Lx*(y + Ly*(z + Lz*t)),  arrays shaped (Lt, Lz, Ly, Lx, ...)

The paper (abstract, section 1) runs MILC's clover_dynamical application on
8x8x16x16 and 16^4 production lattices.  Those gauge configurations are not
available, so random SU(3) fields of the same shapes stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "WORKLOADS",
    "random_su3_field",
    "unit_gauge",
    "random_su3_sites",
    "gauge_transform",
    "pure_gauge",
    "abelian_flux_field",
    "gaussian_source",
    "momenta",
    "heatbath_xi",
    "volume",
]


def volume(dims) -> int:
    lx, ly, lz, lt = dims
    return lx * ly * lz * lt


def _hermitian_traceless(a: np.ndarray) -> np.ndarray:
    h = 0.5 * (a + np.conj(np.swapaxes(a, -1, -2)))
    tr = np.trace(h, axis1=-2, axis2=-1)
    return h - (tr / 3.0)[..., None, None] * np.eye(3)


def _expi_hermitian(h: np.ndarray) -> np.ndarray:
    w, v = np.linalg.eigh(h)
    return (v * np.exp(1j * w)[..., None, :]) @ np.conj(np.swapaxes(v, -1, -2))


def random_su3_field(dims, width: float, seed: int) -> np.ndarray:
    """Links U_mu(x) = exp(i H), H random traceless Hermitian.

    The real and the imaginary part of every entry of a 3x3 complex matrix
    are drawn iid N(0, width^2); the matrix is then Hermitized and made
    traceless.  Links are drawn first from ``default_rng(seed)`` with shape
    (Lt, Lz, Ly, Lx, 4, 3, 3, 2).  Returns complex128 (Lt, Lz, Ly, Lx, 4, 3, 3),
    direction index mu = 0..3 for x, y, z, t.
    """
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((lt, lz, ly, lx, 4, 3, 3, 2))
    a = width * (g[..., 0] + 1j * g[..., 1])
    return _expi_hermitian(_hermitian_traceless(a))


def unit_gauge(dims) -> np.ndarray:
    lx, ly, lz, lt = dims
    u = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1.0
    return u


def random_su3_sites(dims, seed, width: float = 1.0) -> np.ndarray:
    """One random SU(3) matrix per site: complex128 (Lt, Lz, Ly, Lx, 3, 3)."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((lt, lz, ly, lx, 3, 3, 2))
    a = width * (g[..., 0] + 1j * g[..., 1])
    return _expi_hermitian(_hermitian_traceless(a))


def _shift_sites(f: np.ndarray, mu: int) -> np.ndarray:
    """f(x + mu_hat) for a field with site axes (t, z, y, x) first; periodic."""
    return np.roll(f, -1, axis=3 - mu)


def gauge_transform(u: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """U_mu(x) -> Omega(x) U_mu(x) Omega(x+mu)^dagger (a test construction)."""
    out = np.empty_like(u)
    for mu in range(4):
        om_fwd = _shift_sites(omega, mu)
        out[..., mu, :, :] = omega @ u[..., mu, :, :] @ np.conj(np.swapaxes(om_fwd, -1, -2))
    return out


def pure_gauge(dims, seed) -> np.ndarray:
    """U_mu(x) = Omega(x) Omega(x+mu)^dagger: a gauge transform of U = 1."""
    return gauge_transform(unit_gauge(dims), random_su3_sites(dims, seed))


def abelian_flux_field(dims, n: int = 1, embedding: str = "su3") -> np.ndarray:
    """Constant abelian magnetic flux B = 2 pi n / (Lx Ly) through every x-y plaquette.

    With ``embedding="su3"`` the U(1) phase is embedded as
    diag(e^{i th}, e^{-i th}, 1), which keeps every link in SU(3); with
    ``embedding="u1"`` as diag(e^{i th}, 1, 1), a U(3) field whose leaf sum
    has a non-zero trace.  Uses the standard Landau-type gauge for a uniform
    field on a torus: U_y(x) = e^{i B x} everywhere, and U_x(x) = e^{-i B Lx y}
    on the last x slice, so every plaquette carries the same flux B.
    """
    lx, ly, lz, lt = dims
    b = 2.0 * np.pi * n / (lx * ly)
    theta = np.zeros((lt, lz, ly, lx, 4))
    xs = np.arange(lx)[None, None, None, :]
    ys = np.arange(ly)[None, None, :, None]
    theta[..., 1] = np.broadcast_to(b * xs, (lt, lz, ly, lx))
    last = np.zeros((lt, lz, ly, lx))
    last[..., lx - 1] = 1.0
    theta[..., 0] = -b * lx * ys * last
    u = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = np.exp(1j * theta)
    u[..., 1, 1] = np.exp(-1j * theta) if embedding == "su3" else 1.0
    u[..., 2, 2] = 1.0
    return u


def gaussian_source(dims, seed: int, k: int = 0) -> np.ndarray:
    """b(x)_{s,c} = N + iN, iid standard normals, full lattice, from default_rng([seed, 1, k]).

    Returns complex128 (Lt, Lz, Ly, Lx, 4, 3)."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng([seed, 1, k])
    g = rng.standard_normal((lt, lz, ly, lx, 4, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


def momenta(dims, seed: int) -> np.ndarray:
    """Momentum generator coefficients P^a ~ N(0,1), from default_rng([seed, 2]).

    Returns float64 (Lt, Lz, Ly, Lx, 4, 8): one coefficient per Gell-Mann
    generator T^a = lambda^a / 2 per link."""
    lx, ly, lz, lt = dims
    rng = np.random.default_rng([seed, 2])
    return rng.standard_normal((lt, lz, ly, lx, 4, 8))


def heatbath_xi(dims, seed: int) -> np.ndarray:
    """Heat-bath noise on the even checkerboard: re, im ~ N(0, 1/2), so <|xi|^2> = 1.

    From default_rng([seed, 3]).  Returns complex128 (V/2, 4, 3) in even-site
    checkerboard order (even site with lexicographic index i has index i // 2)."""
    vh = volume(dims) // 2
    rng = np.random.default_rng([seed, 3])
    g = rng.standard_normal((vh, 4, 3, 2)) * np.sqrt(0.5)
    return g[..., 0] + 1j * g[..., 1]


@dataclass(frozen=True)
class Workload:
    """One synthetic workload: lattice shape, link roughness and Dirac parameters."""

    name: str
    dims: tuple
    width: float
    kappa: float
    csw: float
    seed: int = 0
    tol: float = 1e-10
    n_sources: int = 1
    t_boundary: int = -1
    notes: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def volume(self) -> int:
        return volume(self.dims)


# The five synthetic workloads: the paper's two lattice shapes (abstract:
# 8x8x16x16 and 16^4), a 4^4 case small enough for dense checks, and a
# 32^3x64 lattice that no longer fits in the GPU's on-die caches.
WORKLOADS = {
    "4^4": Workload("4^4", (4, 4, 4, 4), 0.3, 0.12, 1.0, notes="oracle-sized FP64 solve"),
    "8x8x16x16": Workload("8x8x16x16", (8, 8, 16, 16), 0.5, 0.124, 1.0,
                          notes="FP64 solve + 100 standalone MdagM applications"),
    "16^4": Workload("16^4", (16, 16, 16, 16), 0.3, 0.125, 1.0,
                     notes="FP64 vs mixed CG; fermion force; one HMD step dt=0.02",
                     extra={"dt": 0.02}),
    "32^3x64": Workload("32^3x64", (32, 32, 32, 64), 0.2, 0.1255, 1.0, n_sources=8,
                        notes="mixed vs FP64 CG over 8 sources + force"),
}
