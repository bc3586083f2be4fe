"""Oracle: geometry, gamma matrices, hopping term, clover term, even-odd operators.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain PyTorch CPU,
complex128.

Field shapes (site axes lexicographic, x fastest):
    gauge   U : (Lt, Lz, Ly, Lx, 4, 3, 3)     U[..., mu, a, b], mu = 0..3 for x, y, z, t
    spinor psi: (..., Lt, Lz, Ly, Lx, 4, 3)   any leading batch dims
    eo vector : (..., V/2, 4, 3)              one checkerboard, index i // 2
"""
from __future__ import annotations

import functools

import torch

CDT = torch.complex128
RDT = torch.float64


# ---------------------------------------------------------------- gamma algebra
@functools.lru_cache(maxsize=None)
def _pauli():
    s1 = torch.tensor([[0, 1], [1, 0]], dtype=CDT)
    s2 = torch.tensor([[0, -1j], [1j, 0]], dtype=CDT)
    s3 = torch.tensor([[1, 0], [0, -1]], dtype=CDT)
    return s1, s2, s3


@functools.lru_cache(maxsize=None)
def gammas() -> torch.Tensor:
    """Euclidean gamma matrices in the chiral basis, shape (4, 4, 4), index mu = x, y, z, t.

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = 1, 2, 3 and
    gamma_4 = [[0, 1], [1, 0]] in 2x2 spin blocks.  The paper does not state
    a basis; this one makes gamma_5 diagonal, so the clover term splits into
    two 6x6 blocks on spins {0, 1} and {2, 3}.
    """
    z = torch.zeros(2, 2, dtype=CDT)
    one = torch.eye(2, dtype=CDT)
    out = []
    for s in _pauli():
        out.append(torch.cat([torch.cat([z, -1j * s], 1), torch.cat([1j * s, z], 1)], 0))
    out.append(torch.cat([torch.cat([z, one], 1), torch.cat([one, z], 1)], 0))
    return torch.stack(out)


@functools.lru_cache(maxsize=None)
def gamma5() -> torch.Tensor:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


@functools.lru_cache(maxsize=None)
def sigma_munu() -> torch.Tensor:
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu], shape (4, 4, 4, 4)."""
    g = gammas()
    s = torch.zeros(4, 4, 4, 4, dtype=CDT)
    for mu in range(4):
        for nu in range(4):
            s[mu, nu] = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
    return s


@functools.lru_cache(maxsize=None)
def gell_mann() -> torch.Tensor:
    """The eight Gell-Mann matrices lambda^a, shape (8, 3, 3); generators T^a = lambda^a / 2."""
    lam = torch.zeros(8, 3, 3, dtype=CDT)
    lam[0, 0, 1] = lam[0, 1, 0] = 1
    lam[1, 0, 1], lam[1, 1, 0] = -1j, 1j
    lam[2, 0, 0], lam[2, 1, 1] = 1, -1
    lam[3, 0, 2] = lam[3, 2, 0] = 1
    lam[4, 0, 2], lam[4, 2, 0] = -1j, 1j
    lam[5, 1, 2] = lam[5, 2, 1] = 1
    lam[6, 1, 2], lam[6, 2, 1] = -1j, 1j
    lam[7, 0, 0] = lam[7, 1, 1] = 1 / 3 ** 0.5
    lam[7, 2, 2] = -2 / 3 ** 0.5
    return lam


# ---------------------------------------------------------------- geometry
def lattice_dims(u: torch.Tensor):
    lt, lz, ly, lx = u.shape[:4]
    return (lx, ly, lz, lt)


def parity_mask(dims) -> torch.Tensor:
    """(x + y + z + t) mod 2 on the (Lt, Lz, Ly, Lx) grid (0 = even)."""
    lx, ly, lz, lt = dims
    t = torch.arange(lt).view(lt, 1, 1, 1)
    z = torch.arange(lz).view(1, lz, 1, 1)
    y = torch.arange(ly).view(1, 1, ly, 1)
    x = torch.arange(lx).view(1, 1, 1, lx)
    return (x + y + z + t) % 2


@functools.lru_cache(maxsize=None)
def eo_index(dims):
    """Lexicographic site indices of the even and of the odd sites, in increasing order.

    With Lx even, each pair of sites (2k, 2k+1) holds one site of each parity,
    so the k-th even (odd) site has lexicographic index 2k or 2k+1: the
    checkerboard index of site i is i // 2."""
    par = parity_mask(dims).reshape(-1)
    idx = torch.arange(par.numel())
    return idx[par == 0], idx[par == 1]


def to_eo(psi: torch.Tensor, dims):
    """Full-lattice spinor (..., Lt, Lz, Ly, Lx, 4, 3) -> (even, odd), each (..., V/2, 4, 3)."""
    ev, od = eo_index(tuple(dims))
    flat = psi.reshape(psi.shape[:-6] + (-1, 4, 3))
    return flat[..., ev, :, :], flat[..., od, :, :]


def from_eo(e: torch.Tensor | None, o: torch.Tensor | None, dims) -> torch.Tensor:
    """Inverse of :func:`to_eo`; a missing parity is filled with zeros."""
    lx, ly, lz, lt = dims
    ref = e if e is not None else o
    batch = ref.shape[:-3]
    v = lx * ly * lz * lt
    ev, od = eo_index(tuple(dims))
    flat = torch.zeros(batch + (v, 4, 3), dtype=ref.dtype)
    if e is not None:
        flat = flat.index_copy(len(batch), ev, e)
    if o is not None:
        flat = flat.index_copy(len(batch), od, o)
    return flat.reshape(batch + (lt, lz, ly, lx, 4, 3))


def _site_axis(mu: int) -> int:
    """Axis of direction mu in a spinor (..., Lt, Lz, Ly, Lx, 4, 3)."""
    return -3 - mu


def _gauge_axis(mu: int) -> int:
    """Axis of direction mu in a gauge-like field (Lt, Lz, Ly, Lx, ...)."""
    return 3 - mu


# ---------------------------------------------------------------- hopping term
def hop(u: torch.Tensor, psi: torch.Tensor, t_boundary: float = -1.0, dagger: bool = False) -> torch.Tensor:
    """Wilson hopping term on the full lattice.

    (H psi)(x) = sum_mu eta [ (1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]

    with eta = t_boundary on every hop that crosses the t boundary (both
    directions) and 1 otherwise; x, y, z are periodic.  The adjoint H^dag is
    the same sum with gamma_mu -> -gamma_mu (the gamma matrices are
    Hermitian and the hop to x+mu uses U_mu(x)^dag in H^dag).
    """
    lx, ly, lz, lt = lattice_dims(u)
    g = gammas()
    one = torch.eye(4, dtype=CDT)
    sgn = -1.0 if dagger else 1.0
    out = torch.zeros_like(psi)
    for mu in range(4):
        ax = _site_axis(mu)
        umu = u[..., mu, :, :]
        fwd = torch.roll(psi, -1, dims=ax)  # psi(x + mu)
        bwd = torch.roll(torch.einsum("...ba,...sb->...sa", umu.conj(), psi), 1, dims=ax)  # U(x-mu)^dag psi(x-mu)
        if mu == 3 and t_boundary != 1.0:
            eta_f = torch.ones(lt, dtype=RDT)
            eta_f[lt - 1] = t_boundary
            eta_b = torch.ones(lt, dtype=RDT)
            eta_b[0] = t_boundary
            shape = (lt, 1, 1, 1, 1, 1)
            fwd = fwd * eta_f.view(shape)
            bwd = bwd * eta_b.view(shape)
        fwd = torch.einsum("...ab,...sb->...sa", umu, fwd)
        out = out + torch.einsum("st,...tb->...sb", one - sgn * g[mu], fwd)
        out = out + torch.einsum("st,...tb->...sb", one + sgn * g[mu], bwd)
    return out


# ---------------------------------------------------------------- clover term
def _sh(f: torch.Tensor, mu: int, n: int) -> torch.Tensor:
    """f(x + n mu_hat) for a gauge-like field; periodic (links carry no boundary sign)."""
    return torch.roll(f, -n, dims=_gauge_axis(mu))


def _dag(m: torch.Tensor) -> torch.Tensor:
    return m.conj().transpose(-1, -2)


def clover_leaves(u: torch.Tensor, mu: int, nu: int) -> torch.Tensor:
    """Q_{mu nu}(x): the four plaquettes in the mu-nu plane touching x, all
    traversed counter-clockwise (mu first, then nu) and starting at x."""
    um = u[..., mu, :, :]
    un = u[..., nu, :, :]
    q = um @ _sh(un, mu, 1) @ _dag(_sh(um, nu, 1)) @ _dag(un)
    q = q + un @ _dag(_sh(_sh(um, mu, -1), nu, 1)) @ _dag(_sh(un, mu, -1)) @ _sh(um, mu, -1)
    q = q + _dag(_sh(um, mu, -1)) @ _dag(_sh(_sh(un, mu, -1), nu, -1)) @ _sh(_sh(um, mu, -1), nu, -1) @ _sh(un, nu, -1)
    q = q + _dag(_sh(un, nu, -1)) @ _sh(um, nu, -1) @ _sh(_sh(un, mu, 1), nu, -1) @ _dag(um)
    return q


def clover_field_strength(u: torch.Tensor) -> dict:
    """F_{mu nu}(x) = (Q - Q^dag)/(8i), made traceless; Hermitian 3x3 per site, for mu < nu."""
    eye3 = torch.eye(3, dtype=CDT)
    out = {}
    for mu in range(4):
        for nu in range(mu + 1, 4):
            q = clover_leaves(u, mu, nu)
            f = (q - _dag(q)) / 8j
            tr = torch.diagonal(f, dim1=-2, dim2=-1).sum(-1)
            out[(mu, nu)] = f - (tr / 3)[..., None, None] * eye3
    return out


def clover_matrix(u: torch.Tensor, kappa: float, csw: float) -> torch.Tensor:
    """A(x) = 1 - kappa c_sw sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}(x), shape (Lt, Lz, Ly, Lx, 12, 12).

    Row/column index (s, c) -> 3 s + c.  With this normalisation M = A - kappa H
    equals 2 kappa (D_w + m_0 + c_sw (i/4) sum sigma F) of Luscher, Sint,
    Sommer and Weisz, with the tree-level sign of c_sw."""
    sig = sigma_munu()
    f = clover_field_strength(u)
    shp = u.shape[:4]
    a = torch.eye(12, dtype=CDT).expand(shp + (12, 12)).clone()
    for (mu, nu), fmn in f.items():
        kr = torch.einsum("st,...ab->...satb", sig[mu, nu], fmn).reshape(shp + (12, 12))
        a = a - kappa * csw * kr
    return a


# ---------------------------------------------------------------- operators
class CloverSetup:
    """Gauge field plus the derived clover matrices, and the operators built from them.

    M = A - kappa H on the full lattice.  Even-odd Schur complement on even sites:
        Mhat = A_ee - kappa^2 H_eo A_oo^{-1} H_oe
    """

    def __init__(self, u, kappa: float, csw: float, t_boundary: float = -1.0):
        if not torch.is_tensor(u):
            u = torch.as_tensor(u)
        self.u = u
        self.kappa = float(kappa)
        self.csw = float(csw)
        self.tb = float(t_boundary)
        self.dims = lattice_dims(u)
        lx, ly, lz, lt = self.dims
        assert all(d % 2 == 0 for d in self.dims), "all extents must be even"
        self.V = lx * ly * lz * lt
        self.Vh = self.V // 2
        self.A = clover_matrix(u, kappa, csw)
        ev, od = eo_index(self.dims)
        af = self.A.reshape(self.V, 12, 12)
        self.A_e = af[ev]
        self.A_o = af[od]
        self.Ainv_o = torch.linalg.inv(self.A_o)

    # -- helpers
    @staticmethod
    def _mv(a, psi):
        shp = psi.shape
        return torch.einsum("...ij,...j->...i", a, psi.reshape(shp[:-2] + (12,))).reshape(shp)

    def H(self, psi, dagger=False):
        return hop(self.u, psi, self.tb, dagger)

    def apply_A(self, psi):
        return self._mv(self.A, psi)

    # -- full lattice
    def M(self, psi):
        return self.apply_A(psi) - self.kappa * self.H(psi)

    def Mdag(self, psi):
        return self.apply_A(psi) - self.kappa * self.H(psi, dagger=True)

    # -- even-odd pieces (all vectors are (..., Vh, 4, 3))
    def H_oe(self, e, dagger=False):
        return to_eo(self.H(from_eo(e, None, self.dims), dagger), self.dims)[1]

    def H_eo(self, o, dagger=False):
        return to_eo(self.H(from_eo(None, o, self.dims), dagger), self.dims)[0]

    def Mhat(self, e):
        t = self._mv(self.Ainv_o, self.H_oe(e))
        return self._mv(self.A_e, e) - self.kappa ** 2 * self.H_eo(t)

    def Mhat_dag(self, e):
        """Adjoint A_ee - kappa^2 H_eo^dag A_oo^{-1} H_oe^dag (A and A^{-1} Hermitian)."""
        t = self._mv(self.Ainv_o, self.H_oe(e, dagger=True))
        return self._mv(self.A_e, e) - self.kappa ** 2 * self.H_eo(t, dagger=True)

    def MdagM(self, e):
        return self.Mhat_dag(self.Mhat(e))

    def prepare(self, b_e, b_o):
        """bhat_e = b_e + kappa H_eo A_oo^{-1} b_o."""
        return b_e + self.kappa * self.H_eo(self._mv(self.Ainv_o, b_o))

    def reconstruct(self, x_e, b_o):
        """x_o = A_oo^{-1} (b_o + kappa H_oe x_e)."""
        return self._mv(self.Ainv_o, b_o + self.kappa * self.H_oe(x_e))

    def clover_blocks(self):
        """The two 6x6 chiral blocks of A on every site: (Lt, Lz, Ly, Lx, 2, 6, 6)."""
        return torch.stack([self.A[..., :6, :6], self.A[..., 6:, 6:]], dim=-3)
