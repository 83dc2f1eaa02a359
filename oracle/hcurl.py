"""Nedelec (H(curl)-conforming) space and its mass and curl-curl forms on hexahedra
(oracle; test infrastructure only).

Definitions followed ("Finite Element Discretization": "Finite Elements" for the
H_CURL map type and vector degrees of freedom, "Discrete de Rham Complex" for the
ND spaces; Example 3 of the examples section for the definite Maxwell forms):

* Reference basis of order p >= 1: component a of the vector field is the tensor
  product of the "open" 1D Lagrange basis (p Gauss-Legendre nodes) along axis a
  and the "closed" one (p+1 Gauss-Lobatto nodes) along the other two axes.  The
  dof of basis function (a, i0, i1, i2) is the dot product of the field with the
  unit vector e_a at the node (x_{i0}, x_{i1}, x_{i2}) of that tensor grid: the
  paper's nodal vector dofs r_i . u(node_i) = delta_ij.  3 p (p+1)^2 dofs.
  Local order: component-major, then lexicographic with the first index fastest.
* Map: u(x) = J^{-T} uhat(xhat) (the H_CURL Piola map); its curl maps as
  curl u = J curlhat uhat / det J (curl of an H_CURL function maps with H_DIV).
  For the basis function f(xhat) e_a, curlhat = gradhat f x e_a.
* Element matrices by Gauss quadrature (Q points per direction):
      M_E[i, j] = sum_q w_q beta_q det J (J^{-T} N_i) . (J^{-T} N_j),
      K_E[i, j] = sum_q w_q alpha_q (J C_i) . (J C_j) / det J,
  N the reference values, C the reference curls; J^{-1} from numpy.linalg.inv.
* Global dofs.  A dof is identified without any orientation logic: on the doubled
  index lattice m in [0, 2p]^3 (closed index i -> 2i, open index k -> 2k + 1; the p
  Gauss nodes interlace the p + 1 Lobatto nodes, and the reflection m -> 2p - m maps
  both sets onto themselves), the node of (a, i0, i1, i2) has integer trilinear
  weights prod_b (c_b ? m_b : 2p - m_b) on the eight corners c, and its key is the
  set {(global vertex, weight) : weight > 0}.  Two elements sharing an edge or a
  face produce the same key for the same node.  Nodes of different components
  never coincide (an open index is odd, a closed one even), so the key names the
  dof.  1 / 2 / 4 / 8 non-zero weights never occur / edge / face / interior.
* Global orientation (sign) of a dof, from the global vertex numbers alone: for a
  dof along local axis a, split the corners of its entity (edge, face) into those
  with c_a = 0 and those with c_a = 1; the global basis function points from the
  first group towards the second when the smallest global vertex of the c_a = 1
  group exceeds the smallest of the c_a = 0 group (sign +1), else the local
  function is negated (sign -1).  Interior dofs keep sign +1.  Every element
  sharing the entity agrees, because the two groups are the same vertex sets.
* Essential (tangential) dofs: the dofs of edges and faces of boundary faces.

Pins (tests/test_oracle_hcurl.py): dof counts, the nodal property of the reference
basis, the discrete gradient of the H1 space (each ND dof's value computed from
every element containing it agrees; G^T M G equals the H1 stiffness matrix; the
curl-curl matrix annihilates G), the exact energy of a rotation field on affine
meshes, the null-space dimension of the curl-curl matrix and the definiteness of
the mass matrix by brute force on tiny meshes.
"""
import numpy as np

from .basis import lagrange_derivatives, lagrange_values
from .forms import _jacobians, quadrature_points
from .geometry import lexicographic_corner_slots, map_points
from .quadrature import gauss_legendre, gauss_lobatto


def nd_nodes(p):
    """Closed (p+1 Gauss-Lobatto) and open (p Gauss-Legendre) 1D node sets on [0, 1]."""
    return gauss_lobatto(p + 1), gauss_legendre(p)[0]


def nd_local_index(p):
    """[3 p (p+1)^2, 4] rows (a, i0, i1, i2) in local dof order."""
    rows = []
    for a in range(3):
        n = [p if d == a else p + 1 for d in range(3)]
        for i2 in range(n[2]):
            for i1 in range(n[1]):
                for i0 in range(n[0]):
                    rows.append((a, i0, i1, i2))
    return np.array(rows, dtype=np.int64)


def nd_reference_basis(p, points):
    """Reference values N [npts, ndof, 3] and curls C [npts, ndof, 3] at points [npts, 3]."""
    closed, opened = nd_nodes(p)
    pts = np.asarray(points, dtype=np.float64)
    idx = nd_local_index(p)
    npts, nd = pts.shape[0], idx.shape[0]
    N = np.zeros((npts, nd, 3))
    C = np.zeros((npts, nd, 3))
    tabs = {}
    for kind, nodes in (("c", closed), ("o", opened)):
        for d in range(3):
            tabs[kind, d] = (lagrange_values(nodes, pts[:, d]),
                             lagrange_derivatives(nodes, pts[:, d]))
    for j, (a, i0, i1, i2) in enumerate(idx):
        ii = (i0, i1, i2)
        v, g = [], []
        for d in range(3):
            val, der = tabs["o" if d == a else "c", d]
            v.append(val[:, ii[d]])
            g.append(der[:, ii[d]])
        f = v[0] * v[1] * v[2]
        grad = np.stack([g[0] * v[1] * v[2], v[0] * g[1] * v[2], v[0] * v[1] * g[2]], axis=1)
        N[:, j, a] = f
        e = np.zeros(3)
        e[a] = 1.0
        C[:, j, :] = np.cross(grad, e)
    return N, C


def nd_node_points(p):
    """Reference node [ndof, 3] and direction axis [ndof] of every local dof."""
    closed, opened = nd_nodes(p)
    idx = nd_local_index(p)
    pts = np.empty((idx.shape[0], 3))
    for j, (a, i0, i1, i2) in enumerate(idx):
        ii = (i0, i1, i2)
        for d in range(3):
            pts[j, d] = (opened if d == a else closed)[ii[d]]
    return pts, idx[:, 0].copy()


def _doubled_weights(p):
    """W[j, c]: integer trilinear weights of local dof j's node on lexicographic corner c."""
    idx = nd_local_index(p)
    m = np.empty((idx.shape[0], 3), dtype=np.int64)
    for d in range(3):
        m[:, d] = np.where(idx[:, 0] == d, 2 * idx[:, 1 + d] + 1, 2 * idx[:, 1 + d])
    c = np.arange(8)
    corners = np.stack([c & 1, (c >> 1) & 1, (c >> 2) & 1], axis=1)
    W = np.ones((idx.shape[0], 8), dtype=np.int64)
    for d in range(3):
        W *= np.where(corners[None, :, d] == 1, m[:, None, d], 2 * p - m[:, None, d])
    return W, corners


class NDSpace:
    """Order-p Nedelec space on a hex mesh dict from ``synth`` (trilinear or Q2 geometry)."""

    def __init__(self, mesh: dict, p: int):
        self.mesh = mesh
        self.p = p = int(p)
        if p < 1:
            raise ValueError("Nedelec order must be >= 1")
        hexes = np.asarray(mesh["hex"], dtype=np.int64)
        E = hexes.shape[0]
        V = hexes[:, lexicographic_corner_slots()]                        # [E, 8] lex corners
        W, corners = _doubled_weights(p)
        nd = W.shape[0]
        axis = nd_local_index(p)[:, 0]
        vid = np.where(W[None] > 0, V[:, None, :], -1)                   # [E, nd, 8]
        wts = np.broadcast_to(W[None], vid.shape)
        order = np.argsort(vid, axis=-1, kind="stable")
        svid = np.take_along_axis(vid, order, axis=-1)
        swts = np.take_along_axis(wts, order, axis=-1)
        packed = np.where(svid >= 0, (svid << 16) | swts, -1).reshape(E * nd, 8)
        packed = np.ascontiguousarray(packed)
        row_view = packed.view(np.dtype((np.void, packed.dtype.itemsize * 8))).ravel()
        _, first, inverse = np.unique(row_view, return_index=True, return_inverse=True)
        keys = packed[first]
        cls = (keys >= 0).sum(axis=1)                                    # 2, 4, 8
        assert not np.any(cls == 1), "a Nedelec node on a vertex"
        rank = np.lexsort((first, cls))                                  # edges, faces, interiors
        new_id = np.empty_like(rank)
        new_id[rank] = np.arange(rank.size)
        self.ndofs = int(rank.size)
        self.num_elements = E
        self.elem_dofs = new_id[inverse].reshape(E, nd)
        self.dof_class = cls[rank]
        # orientation: entity corners of each local dof split by c_a
        on = W[None] > 0                                                 # [1, nd, 8]
        side = corners[:, axis].T[None]                                  # [1, nd, 8]: c_a
        big = np.iinfo(np.int64).max
        lo = np.where(on & (side == 0), V[:, None, :], big).min(axis=-1)   # [E, nd]
        hi = np.where(on & (side == 1), V[:, None, :], big).min(axis=-1)
        interior = (W > 0).sum(axis=1) == 8
        self.elem_signs = np.where(interior[None, :], 1.0, np.where(hi > lo, 1.0, -1.0))
        self.boundary = self._boundary_mask(V, W, corners)

    def _boundary_mask(self, V, W, corners):
        """Dofs whose node lies on a boundary face (a face of exactly one element)."""
        E = V.shape[0]
        face_slots = [np.nonzero(corners[:, a] == s)[0] for a in range(3) for s in (0, 1)]
        fkey = np.sort(np.concatenate([V[:, f] for f in face_slots], axis=0), axis=1)
        _, inv, counts = np.unique(fkey, axis=0, return_inverse=True, return_counts=True)
        on_bdr = (counts[inv.ravel()] == 1).reshape(6, E)                  # [face, E]
        mask = np.zeros(self.ndofs, dtype=bool)
        for f, slots in enumerate(face_slots):
            # local dofs whose node lies on face f: every non-zero weight on a face corner
            off = np.setdiff1d(np.arange(8), slots)
            local = np.nonzero((W[:, off] == 0).all(axis=1))[0]
            els = np.nonzero(on_bdr[f])[0]
            mask[self.elem_dofs[np.ix_(els, local)].ravel()] = True
        return mask

    def dof_coordinates(self):
        """Physical node [ndof, 3] of every dof."""
        pts, _ = nd_node_points(self.p)
        x, _ = map_points(self.mesh, pts)                                  # [E, nd, 3]
        out = np.empty((self.ndofs, 3))
        out[self.elem_dofs.ravel()] = x.reshape(-1, 3)
        return out

    def dof_tangents(self):
        """Physical direction [ndof, 3] of every global dof: sign * J e_a at its node."""
        pts, axis = nd_node_points(self.p)
        _, J = map_points(self.mesh, pts)                                  # [E, nd, 3, 3]
        t = np.take_along_axis(J, axis[None, :, None, None].repeat(3, axis=2), axis=3)[..., 0]
        t = t * self.elem_signs[..., None]
        out = np.empty((self.ndofs, 3))
        out[self.elem_dofs.ravel()] = t.reshape(-1, 3)
        return out


def _gram(phys, scale):
    """sum_q scale[e, q] phys[e, q, i, :] . phys[e, q, j, :] for every element, as one
    matrix product per element (rows i against columns j over the (q, component) pairs)."""
    E, nq, nd, _ = phys.shape
    out = np.empty((E, nd, nd))
    for e in range(E):
        F = np.transpose(phys[e], (1, 0, 2)).reshape(nd, 3 * nq)        # [nd, (q, a)]
        out[e] = (F * np.repeat(scale[e], 3)[None, :]) @ F.T
    return out


def element_nd_mass(mesh, p, q1d, coeff=None):
    """Dense element H(curl) mass matrices [E, nd, nd], coefficient None, scalar or [E, Q^3]."""
    pts, w, _, J, det = _jacobians(mesh, q1d)
    N, _ = nd_reference_basis(p, pts)                                     # [Q^3, nd, 3]
    Jinv = np.linalg.inv(J)                                               # [E, Q^3, 3, 3]
    c = 1.0 if coeff is None else np.asarray(coeff)
    scale = np.broadcast_to(w[None, :] * det * c, det.shape)              # [E, Q^3]
    phys = np.einsum("eqba,qjb->eqja", Jinv, N)                           # J^{-T} N
    return _gram(phys, scale)


def element_nd_curlcurl(mesh, p, q1d, coeff=None):
    """Dense element curl-curl matrices [E, nd, nd], coefficient None, scalar or [E, Q^3]."""
    pts, w, _, J, det = _jacobians(mesh, q1d)
    _, C = nd_reference_basis(p, pts)
    c = 1.0 if coeff is None else np.asarray(coeff)
    scale = np.broadcast_to(w[None, :] * c / det, det.shape)
    phys = np.einsum("eqab,qjb->eqja", J, C)                              # J C
    return _gram(phys, scale)


def assemble_nd(space: NDSpace, Ae):
    """Global sparse matrix sum_E S_E G_E^t A_E G_E S_E (S_E the dof signs)."""
    import scipy.sparse as sp
    s = space.elem_signs
    A = Ae * s[:, :, None] * s[:, None, :]
    E, nd = space.elem_dofs.shape
    rows = np.repeat(space.elem_dofs, nd, axis=1).ravel()
    cols = np.tile(space.elem_dofs, (1, nd)).ravel()
    return sp.coo_matrix((A.ravel(), (rows, cols)), shape=(space.ndofs, space.ndofs)).tocsr()


def nd_interpolate(space: NDSpace, field):
    """Dofs of a physical vector field (callable on [..., 3] points): t . u at every node,
    t the global dof direction, taken from every element and checked to agree."""
    pts, axis = nd_node_points(space.p)
    x, J = map_points(space.mesh, pts)
    t = np.take_along_axis(J, axis[None, :, None, None].repeat(3, axis=2), axis=3)[..., 0]
    vals = np.einsum("eja,eja->ej", t, field(x)) * space.elem_signs
    out = np.full(space.ndofs, np.nan)
    out[space.elem_dofs.ravel()] = vals.ravel()
    spread = np.abs(vals - out[space.elem_dofs]).max()
    assert spread < 1e-12 * max(1.0, np.abs(vals).max()), f"inconsistent interpolation {spread}"
    return out


def discrete_gradient(space: NDSpace, h1):
    """Sparse G [nd_dofs, h1_dofs]: the ND dofs of grad phi_h for phi_h in the H1 space of
    the same order on the same mesh, i.e. sign * (d phi_hat / d xhat_a) at each node.

    Returns (G, spread) where spread is the largest disagreement between two elements
    computing the same row (zero for a consistent orientation)."""
    import scipy.sparse as sp
    from .basis import tensor_basis
    pts, axis = nd_node_points(space.p)
    _, grad = tensor_basis(gauss_lobatto(space.p + 1), pts)             # [3, nd, D^3]
    loc = grad[axis, np.arange(axis.size), :]                            # [nd, D^3]
    E = space.num_elements
    rows_l, cols_l, vals_l = [], [], []
    dense = {}
    spread = 0.0
    for e in range(E):
        R = loc * space.elem_signs[e][:, None]
        for j in range(axis.size):
            g = int(space.elem_dofs[e, j])
            row = dict(zip(h1.elem_dofs[e].tolist(), R[j].tolist()))
            if g in dense:
                prev = dense[g]
                ks = set(prev) | set(row)
                spread = max(spread, max(abs(prev.get(k, 0.0) - row.get(k, 0.0)) for k in ks))
            else:
                dense[g] = row
    for g, row in dense.items():
        for h, v in row.items():
            if v != 0.0:
                rows_l.append(g)
                cols_l.append(h)
                vals_l.append(v)
    G = sp.coo_matrix((vals_l, (rows_l, cols_l)), shape=(space.ndofs, h1.ndofs)).tocsr()
    return G, spread
