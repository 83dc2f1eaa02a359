"""Two-dimensional H1 oracle on conforming quadrilateral meshes (test infrastructure only).

The paper's one performance experiment is a 2D Poisson problem ("GPU Acceleration",
the table of 200 partially assembled CG iterations), so the oracle also covers the
2D case with the same definitions as in 3D, restated for quadrilaterals:

* Element map x = sum_i x_{E,i} w_i(xhat), bilinear w_i from the 4 vertices
  ("Meshes / Conforming Meshes", eq. (mesh x)); J_ab = d x_a / d xhat_b.
* Nodal Lagrange basis at the (p+1)^2 Gauss-Lobatto points, lexicographic local
  order i = i1 + (p+1) i2 ("Finite Elements"), evaluated directly in 2D as products
  of 1D Lagrange polynomials (never factorised).
* Global dofs identified topologically without orientation logic: node (i1, i2)
  has integer bilinear weights over the element's four corners,
  w_c = prod_a (c_a ? i_a : p - i_a), and its key is {(vertex id, w_c) : w_c > 0};
  one weight is a vertex dof, two an edge dof, four an interior dof; numbered
  vertices (by vertex id), then edges, then interiors ("Finite Element Spaces").
* Essential dofs: the dofs whose vertices lie on a boundary edge (an edge of one
  element only).
* K_E = sum_q w_q kappa_q det J_q (J_q^-T ghat_i) . (J_q^-T ghat_j) with J^-1 from
  numpy.linalg.inv; M_E = B^T diag(w det J rho) B; b_i = int f phi_i; assembly and
  symmetric elimination reuse :mod:`oracle.forms`.

Pins (tests/test_oracle_2d.py): dof and boundary counts, unit-square element
matrices equal Kronecker products of exact 1D integrals, general affine elements,
K 1 = 0 and 1^T M 1 = area on jittered meshes, the linear patch test, O(h^(p+1)) L2
convergence, invariance under rotated element vertex lists.
"""
import numpy as np

from .basis import lagrange_derivatives, lagrange_values
from .quadrature import gauss_legendre, gauss_lobatto

# quadrilateral vertex slot of lexicographic corner c = cx + 2 cy
_LEX_SLOTS = np.array([0, 1, 3, 2])


def tensor_points_2d(x1d):
    """2D tensor points [n^2, 2], first coordinate fastest."""
    x1d = np.asarray(x1d, dtype=np.float64)
    y, x = np.meshgrid(x1d, x1d, indexing="ij")
    return np.stack([x.ravel(), y.ravel()], axis=1)


def tensor_basis_2d(nodes, points):
    """Values [npts, D^2] and reference gradients [2, npts, D^2] of the 2D basis."""
    nodes = np.asarray(nodes, dtype=np.float64)
    pts = np.asarray(points, dtype=np.float64)
    d1 = nodes.size
    v = [lagrange_values(nodes, pts[:, a]) for a in range(2)]
    g = [lagrange_derivatives(nodes, pts[:, a]) for a in range(2)]
    i2, i1 = np.meshgrid(np.arange(d1), np.arange(d1), indexing="ij")
    i1, i2 = i1.ravel(), i2.ravel()
    val = v[0][:, i1] * v[1][:, i2]
    grad = np.stack([g[0][:, i1] * v[1][:, i2], v[0][:, i1] * g[1][:, i2]])
    return val, grad


def quadrature_points_2d(q1d):
    x, w = gauss_legendre(q1d)
    wy, wx = np.meshgrid(w, w, indexing="ij")
    return tensor_points_2d(x), (wx * wy).ravel()


def map_points_2d(mesh, ref_points):
    """Physical points [E, npts, 2] and Jacobians [E, npts, 2, 2] (bilinear map)."""
    X = np.asarray(mesh["vertices"], dtype=np.float64)[np.asarray(mesh["quad"])[:, _LEX_SLOTS]]
    val, grad = tensor_basis_2d(np.array([0.0, 1.0]), ref_points)
    x = np.einsum("kn,ena->eka", val, X)
    J = np.einsum("bkn,ena->ekab", grad, X)
    return x, J


def _node_weights_2d(p):
    d1 = p + 1
    i2, i1 = np.meshgrid(np.arange(d1), np.arange(d1), indexing="ij")
    idx = np.stack([i1.ravel(), i2.ravel()], axis=1)
    corners = np.array([[0, 0], [1, 0], [0, 1], [1, 1]])
    W = np.ones((idx.shape[0], 4), dtype=np.int64)
    for a in range(2):
        W *= np.where(corners[None, :, a] == 1, idx[:, None, a], p - idx[:, None, a])
    return W


class H1Space2D:
    """Order-p nodal H1 space on a quadrilateral mesh dict from ``synth.quad_lattice``."""

    def __init__(self, mesh, p):
        self.mesh, self.p = mesh, int(p)
        d1 = self.p + 1
        quads = np.asarray(mesh["quad"], dtype=np.int64)
        E = quads.shape[0]
        V = quads[:, _LEX_SLOTS]                                     # [E, 4] lex corners
        W = _node_weights_2d(self.p)                                 # [D^2, 4]
        vid = np.where(W[None] > 0, V[:, None, :], -1)
        wts = np.broadcast_to(W[None], vid.shape)
        order = np.argsort(vid, axis=-1, kind="stable")
        vid = np.take_along_axis(vid, order, axis=-1)
        wts = np.take_along_axis(wts, order, axis=-1)
        packed = np.ascontiguousarray(np.where(vid >= 0, (vid << 12) | wts, -1).reshape(E * d1 ** 2, 4))
        row = packed.view(np.dtype((np.void, packed.dtype.itemsize * 4))).ravel()
        _, first, inverse = np.unique(row, return_index=True, return_inverse=True)
        keys = packed[first]
        cls = (keys >= 0).sum(axis=1)                                # 1, 2, 4
        vkey = np.where(cls == 1, keys.max(axis=1) >> 12, first)
        rank = np.lexsort((vkey, cls))
        new_id = np.empty_like(rank)
        new_id[rank] = np.arange(rank.size)
        self.ndofs = int(rank.size)
        self.elem_dofs = new_id[inverse.ravel()].reshape(E, d1 ** 2)
        self.dof_class = cls[rank]
        keys = keys[rank]
        # boundary edges: vertex pairs of element edges that appear once
        edges = np.concatenate([np.sort(quads[:, [k, (k + 1) % 4]], axis=1) for k in range(4)])
        ue, cnt = np.unique(edges, axis=0, return_counts=True)
        bedges = ue[cnt == 1]
        nv = int(quads.max()) + 1
        bcode = set((bedges[:, 0] * nv + bedges[:, 1]).tolist())
        bverts = np.unique(bedges)
        vs = np.sort(np.where(keys >= 0, keys >> 12, -1), axis=1)   # -1s first
        mask = np.zeros(self.ndofs, dtype=bool)
        c1 = self.dof_class == 1
        mask[c1] = np.isin(vs[c1, 3], bverts)
        c2 = np.nonzero(self.dof_class == 2)[0]
        mask[c2] = [int(a) * nv + int(b) in bcode for a, b in vs[c2, 2:].tolist()]
        self.boundary = mask
        self.num_elements = E

    def dof_coordinates(self):
        x, _ = map_points_2d(self.mesh, tensor_points_2d(gauss_lobatto(self.p + 1)))
        out = np.empty((self.ndofs, 2))
        out[self.elem_dofs.ravel()] = x.reshape(-1, 2)
        return out


def _jacobians_2d(mesh, q1d):
    pts, w = quadrature_points_2d(q1d)
    x, J = map_points_2d(mesh, pts)
    det = np.linalg.det(J)
    if np.any(det <= 0.0):
        raise ValueError("non-positive Jacobian determinant")
    return pts, w, x, J, det


def element_stiffness_2d(mesh, p, q1d, coeff=None):
    """Dense element diffusion matrices [E, D^2, D^2]; coeff None, scalar or [E, Q^2]."""
    from .forms import qpoint_diffusion_operator
    pts, w, _, J, _ = _jacobians_2d(mesh, q1d)
    _, grad = tensor_basis_2d(gauss_lobatto(p + 1), pts)            # [2, Q^2, D^2]
    c = 1.0 if coeff is None else coeff
    Dq = qpoint_diffusion_operator(J, w[None, :], c)                # [E, Q^2, 2, 2]
    H = np.einsum("eqab,bqj->eaqj", Dq, grad)                       # [E, 2, Q^2, D^2]
    return np.einsum("aqi,eaqj->eij", grad, H)


def element_mass_2d(mesh, p, q1d, coeff=None):
    pts, w, _, _, det = _jacobians_2d(mesh, q1d)
    val, _ = tensor_basis_2d(gauss_lobatto(p + 1), pts)
    c = 1.0 if coeff is None else coeff
    d = w[None, :] * det * c
    return np.einsum("qi,eq,qj->eij", val, d, val)


def element_load_2d(mesh, p, q1d, f):
    """Element load vectors [E, D^2]; f callable on points [E, Q^2, 2] or [E, Q^2]."""
    pts, w, x, _, det = _jacobians_2d(mesh, q1d)
    val, _ = tensor_basis_2d(gauss_lobatto(p + 1), pts)
    fq = f(x) if callable(f) else np.asarray(f)
    return np.einsum("qi,eq->ei", val, w[None, :] * det * fq)


def l2_error_2d(space, u_dofs, u_exact, extra=4):
    q = space.p + extra
    pts, w, x, _, det = _jacobians_2d(space.mesh, q)
    val, _ = tensor_basis_2d(gauss_lobatto(space.p + 1), pts)
    uh = np.einsum("qi,ei->eq", val, u_dofs[space.elem_dofs])
    return float(np.sqrt(np.sum(w[None, :] * det * (uh - u_exact(x)) ** 2)))
