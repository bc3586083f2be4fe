"""Shared helpers for the GPU parity tests: seeded inputs on the device, the
oracle's packed clover layout, and error measures."""
import numpy as np
import torch

import oracle as O
from paper_0910_0262_amd import Lattice, synth

C128 = torch.complex128
DEV = "cuda"


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(DEV)


def rel_err(a, b):
    a = torch.as_tensor(a).detach().cpu()
    b = torch.as_tensor(b).detach().cpu()
    return float(torch.linalg.norm((a - b).reshape(-1)) / torch.linalg.norm(b.reshape(-1)))


def max_rel(a, b):
    a = torch.as_tensor(a).detach().cpu()
    b = torch.as_tensor(b).detach().cpu()
    return float(torch.abs(a - b).max() / torch.abs(b).max())


def pack_blocks(a12: torch.Tensor) -> torch.Tensor:
    """Oracle 12x12 clover matrices (..., 12, 12) -> packed (..., 2, 36) float64."""
    out = []
    for b in range(2):
        blk = a12[..., 6 * b:6 * b + 6, 6 * b:6 * b + 6]
        d = torch.diagonal(blk, dim1=-2, dim2=-1).real
        iu = torch.triu_indices(6, 6, 1)
        off = blk[..., iu[0], iu[1]]
        out.append(torch.cat([d, torch.stack([off.real, off.imag], -1).reshape(off.shape[:-1] + (30,))], -1))
    return torch.stack(out, -2)


def make_case(dims, width, kappa, csw, seed=0, t_boundary=-1, field="random"):
    if field == "random":
        u = synth.random_su3_field(dims, width, seed)
    elif field == "unit":
        u = synth.unit_gauge(dims)
    else:
        raise ValueError(field)
    lat = Lattice(dims, kappa, csw, t_boundary)
    ud = to_dev(u)
    lat.load_gauge(ud)
    setup = O.CloverSetup(torch.as_tensor(u), kappa, csw, t_boundary)
    return lat, setup, u, ud


def random_spinor(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape + (4, 3)) + 1j * rng.standard_normal(shape + (4, 3))
