"""MI355X (gfx950) even-odd Wilson-clover solver and fermion force.

The hot path of the dynamical clover-fermion HMD (R algorithm) application
studied in arXiv:0910.0262: the even-odd preconditioned Wilson-clover
operator, CG on Mhat^dag Mhat in FP64 or mixed precision with reliable
updates, and the fermion force, implemented as HIP kernels behind the C ABI
in include/cloverqcd.h.  ``capi`` mirrors the C entry points one to one;
``Lattice`` and ``CloverForce`` are thin conveniences over it.
"""
from .lattice import CloverForce, Lattice, QCDError  # noqa: F401

__all__ = ["Lattice", "CloverForce", "QCDError"]
