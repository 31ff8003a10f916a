"""Seeded synthetic inputs shared by the tests, the bench and the oracle.

This package only *builds inputs* (sparse matrices in CSR form, the random
perturbation diagonal D and the Gaussian start block Omega).  It holds none of
the null-space method's arithmetic: it never applies the operator, never
orthogonalises and never computes a null-space basis.  Construction metadata
(component labels, the planted coupling matrix R) is returned so that the
oracle can write down the exact null space itself.
"""
from .generators import (  # noqa: F401
    CSR,
    er_component_laplacian,
    planted_nullity,
    rgg_coboundary,
    zipf_component_laplacian,
    fd_instance,
    perturbation_diagonal,
    gaussian_start_block,
    gaussian_matrix,
    config,
)
