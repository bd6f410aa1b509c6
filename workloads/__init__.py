"""Seeded synthetic inputs for the SIPDG monodomain solver.

This package produces *problem data only*: vertex coordinates and cell
connectivity of quadrilateral/hexahedral meshes, per-cell conductivity
tensors, initial values at DoF nodes, stimulus masks and sensor sets.  It
contains none of the method's arithmetic (no basis functions used for
assembly, no quadrature, no operators, no solvers).  Both the independent
CPU oracle and the GPU library consume these arrays; nothing here is shared
beyond the inputs themselves.
"""
from .meshes import structured_mesh, cell_centroids, dof_nodes, gl_nodes_1d
from .configs import CONFIGS, make_problem

__all__ = ["structured_mesh", "cell_centroids", "dof_nodes", "gl_nodes_1d",
           "CONFIGS", "make_problem"]
