"""Seeded synthetic problem generators shared by the GPU path and the oracle.

This package builds meshes, permeability fields, boundary data and sources.
It holds none of the solver's arithmetic: no transmissibilities, no
residuals, no coarsening.  Every array it returns is plain geometry or data
of the boundary-value problem of Section 2 (mass conservation + Darcy's law
with K(x, p) = K0(x) kappa(p), Dirichlet and Neumann boundary data).
"""
from .grids import (Mesh, Problem, cartesian_mesh, c1_problem, c2_problem,
                    small_problem, permute_mesh, gaussian_field, channel_field)

__all__ = ["Mesh", "Problem", "cartesian_mesh", "c1_problem", "c2_problem",
           "small_problem", "permute_mesh", "gaussian_field", "channel_field"]
