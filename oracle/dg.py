"""Discontinuous (L2) space and the upwind DG convection form on hexahedra (oracle;
test infrastructure only).

Definitions followed ("Finite Element Discretization": L2 elements among the de Rham
spaces, "Discrete de Rham Complex"; convection "including DG" among the partially
assembled integrators of "GPU Acceleration"; the DG advection of the examples section):

* Space: on every element the nodal Lagrange basis on the (p+1)^3 Gauss-Lobatto
  points, with no continuity between elements; dof e * (p+1)^3 + i, i lexicographic.
* Operator of the steady transport term div(beta u) with a constant velocity beta,
  upwind fluxes and zero inflow data:
      a(u, v) = - sum_K int_K u (beta . grad v)
                + sum_{interior F} int_F (beta . n) u_up (v^- - v^+)
                + int_{outflow part of dOmega} (beta . n) u v,
  n the unit normal of F pointing from its element "-" to its element "+", u_up the
  trace from the element the flow leaves (u^- where beta . n > 0, else u^+).  On an
  element the volume term is minus the transpose of the H1 convection matrix of the
  same element (oracle.forms.element_convection).  Face integrals use the tensor Gauss
  rule with q1d points per direction on the "-" side's reference face; the "+" side
  evaluates its basis at the same physical points, found through the two faces'
  shared corners (the map between the two reference faces is the symmetry of the
  square that carries one corner labelling to the other).  The area-weighted normal
  is the cross product of the two tangent vectors of the "-" side's face map.

Pins (tests/test_oracle_dg.py): on affine meshes, a(u, w) for piecewise-linear
discontinuous u and w equals the same integrals evaluated directly in physical space
(no reference element, no face matching); the constant field is mapped to the inflow
boundary flux alone; restricted to continuous fields and test functions vanishing on
the inflow boundary, the form equals the H1 convection form; a(u, u) is non-negative.
"""
import numpy as np
import scipy.sparse as sp

from .basis import tensor_basis
from .forms import element_convection
from .geometry import element_geometry_nodes, lexicographic_corner_slots
from .quadrature import gauss_legendre, gauss_lobatto


def _faces(mesh):
    """Interior faces [(e-, f-, e+, f+)] and boundary faces [(e, f)]; f = 2 a + side."""
    V = np.asarray(mesh["hex"], dtype=np.int64)[:, lexicographic_corner_slots()]
    E = V.shape[0]
    c = np.arange(8)
    corners = np.stack([c & 1, (c >> 1) & 1, (c >> 2) & 1], axis=1)
    seen = {}
    interior, boundary = [], []
    for e in range(E):
        for a in range(3):
            for side in (0, 1):
                f = 2 * a + side
                key = tuple(sorted(V[e, corners[:, a] == side].tolist()))
                if key in seen:
                    e0, f0 = seen.pop(key)
                    interior.append((e0, f0, e, f))
                else:
                    seen[key] = (e, f)
    boundary = sorted(seen.values())
    return interior, boundary, V, corners


def _face_ref_points(f, st):
    """Reference points [n, 3] of face f at face coordinates st [n, 2] (the two
    tangential axes in increasing order)."""
    a, side = divmod(f, 2)
    b, cax = [d for d in range(3) if d != a]
    out = np.empty((st.shape[0], 3))
    out[:, a] = side
    out[:, b] = st[:, 0]
    out[:, cax] = st[:, 1]
    return out


def _map(X, gnodes, ref):
    """Physical points [n, 3] and Jacobians [n, 3, 3] of one element at reference points."""
    val, grad = tensor_basis(gnodes, ref)
    return val @ X, np.einsum("bkn,na->kab", grad, X)


def _plus_side_points(Vm, fm, Vp, fp, st, corners):
    """Reference points on face fp of the '+' element matching face coordinates st of
    face fm of the '-' element (through the shared corner vertex ids)."""
    am, sm = divmod(fm, 2)
    bm, cm = [d for d in range(3) if d != am]
    ap, sp_ = divmod(fp, 2)
    ref_of_vertex = {}
    for k in range(8):
        if corners[k, ap] == sp_:
            ref_of_vertex[int(Vp[k])] = corners[k].astype(float)
    def corner_at(s, t):
        for k in range(8):
            if corners[k, am] == sm and corners[k, bm] == s and corners[k, cm] == t:
                return ref_of_vertex[int(Vm[k])]
        raise AssertionError("corner not found")
    C00, C10, C01 = corner_at(0, 0), corner_at(1, 0), corner_at(0, 1)
    return C00[None] + st[:, :1] * (C10 - C00)[None] + st[:, 1:] * (C01 - C00)[None]


def _outward_normal(J, f):
    """Area-weighted outward normal of face f from Jacobians J [n, 3, 3]."""
    a, side = divmod(f, 2)
    b, cax = [d for d in range(3) if d != a]
    N = np.cross(J[:, :, b], J[:, :, cax])
    perm_sign = 1.0 if (a, b, cax) in ((0, 1, 2), (1, 2, 0), (2, 0, 1)) else -1.0
    return N * perm_sign * (1.0 if side == 1 else -1.0)


class DGSpace:
    """Order-p discontinuous nodal space (Gauss-Lobatto nodes) on a hex mesh dict."""

    def __init__(self, mesh: dict, p: int):
        self.mesh, self.p = mesh, int(p)
        E = mesh["hex"].shape[0]
        self.num_elements = E
        self.dpe = (self.p + 1) ** 3
        self.ndofs = E * self.dpe
        self.elem_dofs = np.arange(self.ndofs).reshape(E, self.dpe)


def dg_convection_matrix(mesh, p, q1d, beta):
    """Global sparse matrix of a(u, v) above (row = test dof, column = trial dof)."""
    beta = np.asarray(beta, dtype=np.float64)
    E = mesh["hex"].shape[0]
    D3 = (p + 1) ** 3
    nodes = gauss_lobatto(p + 1)
    rows, cols, vals = [], [], []

    def add(block, ei, ej):
        ri = np.repeat(np.arange(D3) + ei * D3, D3)
        cj = np.tile(np.arange(D3) + ej * D3, D3)
        rows.append(ri)
        cols.append(cj)
        vals.append(block.ravel())

    C = element_convection(mesh, p, q1d, beta)                         # [E, test, trial]
    for e in range(E):
        add(-C[e].T, e, e)
    interior, boundary, V, corners = _faces(mesh)
    X, gn = element_geometry_nodes(mesh)
    x1, w1 = gauss_legendre(q1d)
    T, S = np.meshgrid(x1, x1, indexing="ij")
    st = np.stack([S.ravel(), T.ravel()], axis=1)                      # s fastest
    wq = np.outer(w1, w1).ravel()
    for (em, fm, ep, fp) in interior:
        rm = _face_ref_points(fm, st)
        _, Jm = _map(X[em], gn, rm)
        bn = wq * (_outward_normal(Jm, fm) @ beta)                      # w beta . N
        rp = _plus_side_points(V[em], fm, V[ep], fp, st, corners)
        phim, _ = tensor_basis(nodes, rm)                               # [nq, D3]
        phip, _ = tensor_basis(nodes, rp)
        up_minus = bn > 0
        # u_up = u^- where beta . n > 0, u^+ elsewhere; tested with v^- - v^+
        wm = np.where(up_minus, bn, 0.0)
        wp = np.where(up_minus, 0.0, bn)
        add(phim.T @ (wm[:, None] * phim), em, em)
        add(-(phip.T @ (wm[:, None] * phim)), ep, em)
        add(phim.T @ (wp[:, None] * phip), em, ep)
        add(-(phip.T @ (wp[:, None] * phip)), ep, ep)
    for (e, f) in boundary:
        r = _face_ref_points(f, st)
        _, J = _map(X[e], gn, r)
        bn = wq * (_outward_normal(J, f) @ beta)
        phi, _ = tensor_basis(nodes, r)
        wo = np.where(bn > 0, bn, 0.0)                                  # outflow only
        add(phi.T @ (wo[:, None] * phi), e, e)
    n = E * D3
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def dg_node_coordinates(mesh, p):
    """Physical node [E * (p+1)^3, 3] of every DG dof."""
    from .basis import tensor_points
    from .geometry import map_points
    x, _ = map_points(mesh, tensor_points(gauss_lobatto(p + 1)))
    return x.reshape(-1, 3)
