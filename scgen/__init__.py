"""Seeded synthetic FETI subdomains: structured-grid FEM stiffness, kernel basis,
regularisation and the signed-boolean gluing matrix B.

This module produces INPUTS only.  It holds none of the Schur-complement
method's arithmetic (no ordering, no factorisation, no triangular solve, no
product with B): both the product path and the test oracle consume what it
returns, and it imports neither of them.

Problem statement (paper, Sec. 2.1, eqs. (1)-(9)):
  * K_i  -- sparse SPSD subdomain stiffness of a floating subdomain (no
    Dirichlet condition), here heat transfer (1 DOF per node) or isotropic
    linear elasticity (3 DOFs per node) on a box of bilinear (Q1, 2D) or
    trilinear (hex8, 3D) elements;
  * R_i  -- basis of Ker K_i (constant vector / six rigid-body modes);
  * K_reg -- the regularised matrix whose inverse is a generalised inverse of
    K_i (Sec. 2.2, eq. (10)); obtained here by the fixing-node regularisation
    that the paper cites: K_reg = K + rho * Q Q^T with Q an orthonormal basis
    of R restricted to a few fixing DOFs.  Any Q with Q^T R nonsingular gives
    K K_reg^{-1} K = K;
  * B_i  -- signed boolean: column j of B^T has a single entry sign_j at row
    dof_j (one Lagrange multiplier per glued surface DOF).
"""
from .mesh import (Subdomain, heat_q1_2d, heat_hex8, elasticity_hex8, laplace_1d,
                   box_subdomain)
from .simplex import simplex_subdomain, p1_stiffness
from .rng import splitmix64, splitmix64_uniform
from .configs import (config_subdomains, CONFIG_NAMES, BASE_SEED, config_description,
                      uneven_sizes, paper_subdomains, paper_batch_size, PAPER_NODES)

__all__ = [
    "Subdomain", "heat_q1_2d", "heat_hex8", "elasticity_hex8", "laplace_1d",
    "box_subdomain", "simplex_subdomain", "p1_stiffness", "splitmix64", "splitmix64_uniform", "config_subdomains",
    "CONFIG_NAMES", "BASE_SEED", "config_description", "uneven_sizes", "paper_subdomains",
    "paper_batch_size", "PAPER_NODES",
]
