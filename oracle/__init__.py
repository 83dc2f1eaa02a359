"""Plain CPU FP64 oracle for the H1 diffusion / mass partial-assembly path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The GPU library never
calls it, and it shares no code with the GPU library: it assembles global sparse
matrices from dense element matrices (no sum factorization, no partial
assembly) exactly as the weak form defines them, and solves with a textbook
preconditioned CG.

Citations refer to the MFEM paper (arXiv:1911.09220) by section / equation:

* Model problem and weak form: "Finite Element Abstractions", eq. (strong
  Poisson), eq. (weak Poisson), eq. (abstract forms), eq. (linear system).
* Mesh map x = sum_i x_{E,i} w_i(xhat): "Meshes / Conforming Meshes", eq. (mesh x).
* Nodal H1 basis at Gauss-Lobatto points, local dof order, global numbering
  vertices -> edges -> faces -> interiors: "Finite Element Discretization",
  subsections "Finite Elements" and "Finite Element Spaces".
* Element mass matrix by quadrature, M_E = B^t D_E B: "High-Order Partial
  Assembly", the mass-matrix equations.
* FormLinearSystem with essential boundary conditions: "Finite Element Linear
  Systems".
* CG on the operator: "Scalable Linear Solvers" (ex1p listing).

Every function here is pinned by tests under ``tests/`` (closed forms,
invariants, brute force, convergence rates), see the module docstrings.
"""
from .quadrature import gauss_legendre, gauss_lobatto
from .basis import lagrange_values, lagrange_derivatives, tensor_basis
from .geometry import element_geometry_nodes, map_points
from .space import H1Space
from .forms import (qpoint_diffusion_operator, element_stiffness, element_mass,
                    element_load, assemble, constrain, quadrature_points)
from .solvers import pcg, l2_error

__all__ = [
    "gauss_legendre", "gauss_lobatto", "lagrange_values", "lagrange_derivatives",
    "tensor_basis", "element_geometry_nodes", "map_points", "H1Space",
    "qpoint_diffusion_operator", "element_stiffness", "element_mass", "element_load",
    "assemble", "constrain", "quadrature_points", "pcg", "l2_error",
]
