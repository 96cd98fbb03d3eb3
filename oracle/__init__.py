"""CPU FP64 reference for the high-contrast elasticity state solve.

TEST INFRASTRUCTURE ONLY.  This package is the oracle that the GPU library is
checked against.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import it; the product path never does.

It is written for a reader who has the paper (Zambrano, Serrano, Lazarov,
Galvis, "Fast multiscale contrast independent preconditioners for linear
elastic topology optimization problems", arXiv:2006.13387) beside it.  It
computes, plainly and slowly, in float64:

* SIMP moduli (Section 1, the SIMP interpolation law);
* Q1 (2D plane stress) / trilinear H8 (3D) element stiffness with C = E C0
  (Section 1.1, Navier-Cauchy problem, its weak form and bilinear
  discretisation) and global sparse assembly of K(rho);
* the overlapping subdomains D'_i and the first level
  sum_i R_i^T K_i^{-1} R_i (Section 2, overlapping decomposition and the
  two-level additive preconditioner);
* the heat (scalar diffusion) eigenproblems on coarse neighbourhoods with an
  eigenvalue threshold (Section 4.1), the component-wise coarse space V_0,H
  and its rotation enrichment (Section 4.2);
* the preconditioner M_EH+Rot, and M_EH without rotations (Section 4.3,
  Table 1);
* PCG and the Lanczos condition estimate (Section 2 and Section 5);
* the density gradient of the compliance (or of l^T u through an adjoint)
  and one optimality-criteria design update (Section 1), in ``topopt``.

Functions pinned by no independent check say "parity unpinned" in their
docstring.  At the time of writing every function here has a pin in
``tests/test_oracle_*.py``.
"""
from .fem import (simp_modulus, elasticity_element, heat_element,
                  assemble_stiffness, assemble_scalar, element_node_ids,
                  node_coords, rigid_body_modes)
from .dd import (Hierarchy, subdomain_node_boxes, coarse_node_grid,
                 neighbourhood, partition_of_unity, heat_pencil, heat_modes,
                 build_coarse_basis, build_preconditioner)
from .pcg import pcg, lanczos_condition
from .solve import solve, direct_solve, reference_solution

__all__ = [
    "simp_modulus", "elasticity_element", "heat_element", "assemble_stiffness",
    "assemble_scalar", "element_node_ids", "node_coords", "rigid_body_modes",
    "Hierarchy", "subdomain_node_boxes", "coarse_node_grid", "neighbourhood",
    "partition_of_unity", "heat_pencil", "heat_modes", "build_coarse_basis",
    "build_preconditioner", "pcg", "lanczos_condition", "solve",
    "direct_solve", "reference_solution",
]
