"""H1 finite element space on a conforming hexahedral mesh (oracle; test infrastructure only).

"Finite Element Discretization / Finite Element Spaces": the space stores, per
element, the ordered list of global dof indices; global dofs are numbered all
vertex dofs first, then edge, face and interior dofs.  Shared edge/face dofs
must be identified consistently by all neighbouring elements regardless of each
element's local orientation ("Finite Elements", orientation permutations of
FiniteElementCollection).

The oracle identifies a dof *topologically and without any orientation logic*:
the node with lexicographic index (i1, i2, i3) in [0, p]^3 has integer
trilinear weights over the element's eight corners,
    w_c = prod_a (c_a ? i_a : p - i_a),
and the key of the dof is the set {(global vertex id, w_c) : w_c > 0}.  Two
elements sharing an entity produce the same key for the same node whatever their
vertex order.  The number of non-zero weights classifies the dof (1 vertex,
2 edge, 4 face, 8 interior), which gives the paper's numbering order.

Boundary (essential) dofs are the dofs whose vertex set lies in a boundary face,
a face belonging to exactly one element.

Pins: dof counts (n p + 1)^3, boundary counts, numbering-invariance of the
assembled operator under random element rotations (tests/test_oracle_space.py).
"""
import numpy as np

from .basis import tensor_points
from .geometry import lexicographic_corner_slots, map_points
from .quadrature import gauss_lobatto


def _lex_corners():
    c = np.arange(8)
    return np.stack([c & 1, (c >> 1) & 1, (c >> 2) & 1], axis=1)


def _node_weights(p):
    """W[i, c] integer trilinear weights of local node i on lexicographic corner c."""
    d1 = p + 1
    i3, i2, i1 = np.meshgrid(np.arange(d1), np.arange(d1), np.arange(d1), indexing="ij")
    idx = np.stack([i1.ravel(), i2.ravel(), i3.ravel()], axis=1)        # [D^3, 3]
    corners = _lex_corners()                                            # [8, 3]
    W = np.ones((idx.shape[0], 8), dtype=np.int64)
    for a in range(3):
        W *= np.where(corners[None, :, a] == 1, idx[:, None, a], p - idx[:, None, a])
    return W


class H1Space:
    """Order-p nodal H1 space (Gauss-Lobatto nodes) on a hex mesh dict from ``synth``."""

    def __init__(self, mesh: dict, p: int):
        self.mesh = mesh
        self.p = p = int(p)
        d1 = p + 1
        hexes = np.asarray(mesh["hex"], dtype=np.int64)
        E = hexes.shape[0]
        V = hexes[:, lexicographic_corner_slots()]                       # [E, 8] lex corners
        W = _node_weights(p)                                            # [D^3, 8]
        vid = np.where(W[None, :, :] > 0, V[:, None, :], -1)            # [E, D^3, 8]
        wts = np.broadcast_to(W[None, :, :], vid.shape)
        order = np.argsort(vid, axis=-1, kind="stable")
        vid = np.take_along_axis(vid, order, axis=-1)
        wts = np.take_along_axis(wts, order, axis=-1)
        packed = np.where(vid >= 0, (vid << 12) | wts, -1).reshape(E * d1 ** 3, 8)
        packed = np.ascontiguousarray(packed)
        row_view = packed.view(np.dtype((np.void, packed.dtype.itemsize * 8))).ravel()
        _, first, inverse = np.unique(row_view, return_index=True, return_inverse=True)
        keys = packed[first]                                            # [ndof, 8]
        cls = (keys >= 0).sum(axis=1)                                   # 1, 2, 4, 8
        # vertex dofs by vertex id, the other classes by first appearance
        vkey = np.where(cls == 1, keys.max(axis=1) >> 12, first)
        rank = np.lexsort((vkey, cls))
        new_id = np.empty_like(rank)
        new_id[rank] = np.arange(rank.size)
        self.ndofs = int(rank.size)
        self.elem_dofs = new_id[inverse].reshape(E, d1 ** 3)
        self.dof_class = cls[rank]
        self._keys = keys[rank]
        self.boundary = self._boundary_mask(V)
        self.num_elements = E

    def _boundary_mask(self, V):
        corners = _lex_corners()
        nv = int(V.max()) + 1
        face_slots = [np.nonzero(corners[:, a] == side)[0] for a in range(3) for side in (0, 1)]
        fv = np.concatenate([V[:, f] for f in face_slots], axis=0)            # [6E, 4]
        fkey = np.sort(fv, axis=1)
        _, inv, counts = np.unique(fkey, axis=0, return_inverse=True, return_counts=True)
        on_bdr = counts[inv.ravel()] == 1                                     # [6E]
        bfaces = set(map(tuple, fkey[on_bdr].tolist()))
        bverts = np.unique(fkey[on_bdr])
        # edges of a face: corner pairs that differ in exactly one coordinate
        fc = corners[face_slots[0]]
        pairs = [(i, j) for i in range(4) for j in range(i + 1, 4)
                 if np.abs(fc[i] - fc[j]).sum() == 1]
        bdr_fv = fv[on_bdr]
        edge_codes = []
        for (i, j) in pairs:
            a, b = bdr_fv[:, i], bdr_fv[:, j]
            edge_codes.append(np.minimum(a, b) * nv + np.maximum(a, b))
        bedges = np.unique(np.concatenate(edge_codes))
        vs = np.where(self._keys >= 0, self._keys >> 12, -1)
        vs = np.sort(vs, axis=1)                                             # -1s first
        mask = np.zeros(self.ndofs, dtype=bool)
        c1 = self.dof_class == 1
        mask[c1] = np.isin(vs[c1, 7], bverts)
        c2 = self.dof_class == 2
        mask[c2] = np.isin(vs[c2, 6] * nv + vs[c2, 7], bedges)
        c4 = np.nonzero(self.dof_class == 4)[0]
        mask[c4] = [tuple(r) in bfaces for r in vs[c4, 4:].tolist()]
        return mask

    def dof_coordinates(self):
        """Physical position [ndof, 3] of every dof node."""
        nodes = gauss_lobatto(self.p + 1)
        x, _ = map_points(self.mesh, tensor_points(nodes))            # [E, D^3, 3]
        coords = np.empty((self.ndofs, 3))
        coords[self.elem_dofs.ravel()] = x.reshape(-1, 3)
        return coords

    def boundary_dofs(self):
        return np.nonzero(self.boundary)[0]
