"""Element maps x = Phi(xhat) and Jacobians (oracle; test infrastructure only).

"Meshes / Conforming Meshes", eq. (mesh x): x(xhat) = sum_i x_{E,i} w_i(xhat),
with trilinear w_i from the 8 vertices, or a nodal description with more nodes
per element (here 27 nodes of a quadratic map at {0, 1/2, 1}^3).  The Jacobian is
J_ab = d x_a / d xhat_b, obtained by differentiating the same expansion.

Pins: volume = sum_q w_q det J_q = 1 on jittered unit cubes, affine maps give
constant J, orientation-preserving relabelling leaves det J > 0
(tests/test_oracle_forms.py).
"""
import numpy as np

from .basis import tensor_basis

# Reference corner of each slot of the usual hexahedron vertex order.
_HEX_CORNER = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                        [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]])


def lexicographic_corner_slots():
    """slot[c] = hexahedron vertex slot of lexicographic corner c = cx + 2cy + 4cz."""
    out = np.empty(8, dtype=np.int64)
    for s, (cx, cy, cz) in enumerate(_HEX_CORNER):
        out[cx + 2 * cy + 4 * cz] = s
    return out


def element_geometry_nodes(mesh: dict):
    """Per-element geometry nodes [E, ng, 3] (lexicographic) and the node set in 1D."""
    if mesh.get("geom_order", 1) == 1 or mesh.get("geom_nodes") is None:
        slots = lexicographic_corner_slots()
        X = mesh["vertices"][mesh["hex"][:, slots]]
        return X, np.array([0.0, 1.0])
    return np.asarray(mesh["geom_nodes"], dtype=np.float64), np.array([0.0, 0.5, 1.0])


def map_points(mesh: dict, ref_points):
    """Physical points [E, npts, 3] and Jacobians [E, npts, 3, 3] at reference points."""
    X, gnodes = element_geometry_nodes(mesh)
    val, grad = tensor_basis(gnodes, ref_points)               # [npts, ng], [3, npts, ng]
    x = np.einsum("kn,ena->eka", val, X)
    J = np.einsum("bkn,ena->ekab", grad, X)
    return x, J
