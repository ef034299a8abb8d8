"""FP64 CPU oracle for Progressively Projected Newton (PPN) and its comparison modes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU library
(no kernels, headers, tables or helpers); both sides take their inputs from
the separate ``scenes`` input generator.

The oracle is written to be checked by eye against the paper
(arXiv 2505.21013, "Progressively Projected Newton"):

* ``snh``      Stable Neo-Hookean energy density and its first and second
               derivatives with respect to F (Sec. 5.1, material model).
* ``fem``      linear-tetrahedron kinematics, element energy / gradient /
               Hessian, lumped mass and the backward-Euler incremental
               potential (Sec. 3, Eq. (1); Sec. 5.1 time stepping).
* ``assemble`` additive global assembly H = sum_e H^e, g = sum_e g^e (Sec. 3).
* ``project``  eigenvalue clamping of an element Hessian (Sec. 3, Eq. (4)).
* ``pcg``      block-Jacobi PCG that reports indefiniteness (Sec. 4.1).
* ``newton``   one time step by PN, PDN or PPN (Algorithm 1, Sec. 4 and 5.1).

Everything is single-threaded NumPy / SciPy in float64.  Every function is a
plain definition or the algorithm's steps in the paper's order; no blocking or
fusion beyond a loop over element chunks that only bounds memory.

Readings of points the paper leaves open are listed in the docstring of
``newton`` and in the comments of the functions that implement them.
"""
from .snh import lame_to_snh, psi, first_piola, d2psi_dF2
from .fem import Mesh, element_psi, element_grad_hess, lumped_mass
from .project import project_to_pd
from .pcg import pcg_block_jacobi
from .newton import Params, Stepper, run_scene

__all__ = [
    "lame_to_snh", "psi", "first_piola", "d2psi_dF2",
    "Mesh", "element_psi", "element_grad_hess", "lumped_mass",
    "project_to_pd", "pcg_block_jacobi", "Params", "Stepper", "run_scene",
]
