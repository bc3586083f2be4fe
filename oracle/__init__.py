"""CPU oracle for the even-odd Wilson-clover solve and fermion force.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library,
its Python binding, the benchmark's timed GPU legs) imports, links or calls
anything here.  Only the tests, the smoke check and the benchmark's CPU
baseline leg use it.  It shares no code, header, table or constant with the
HIP implementation.

It is written in plain PyTorch CPU operations in complex128 (FP64), chosen
for obviousness over speed: whole-lattice ``torch.roll`` shifts, dense 4x4
gamma matrices, dense 12x12 clover matrices, textbook conjugate gradient, and
autograd of the operator for the force.

The paper (Shi, Kindratenko, Gottlieb, arXiv:0910.0262, abstract and section
1) names the computation -- MILC clover_dynamical with dynamical clover
fermions and the hybrid-molecular-dynamics R algorithm -- but prints no
equation.  Every definition below is therefore the textbook one, with the
conventions written out in each function and listed in the design notes:
Wilson-clover operator in hopping form after Luscher, Sint, Sommer and Weisz
(Nucl. Phys. B478 (1996) 365), a chiral Euclidean gamma basis, even-odd
(Schur complement) preconditioning, CG (Hestenes-Stiefel) on the normal
equations, and the HMD update of the R algorithm (the step schedule of
Gottlieb, Liu, Toussaint, Renken and Sugar, Phys. Rev. D 35 (1987) 2531).
"""
from .core import (  # noqa: F401
    CloverSetup,
    gammas,
    gamma5,
    sigma_munu,
    gell_mann,
    hop,
    clover_field_strength,
    clover_matrix,
    parity_mask,
    eo_index,
    to_eo,
    from_eo,
)
from .solve import cg, solve_full, dense_matrix  # noqa: F401
from .force import action, action_and_gradient, project_force, action_variational  # noqa: F401
from .hmd import expi_su3, r_step, hmd_step, hamiltonian  # noqa: F401
from .quant import quantize16, dequantize16, link_to_half12, reconstruct12  # noqa: F401
from . import md  # noqa: F401
