"""Helpers shared by the tests: oracle problem setup and dof matching by position.

The library and the oracle number dofs differently; results are compared after
matching dofs by their node coordinates (each H1 dof has a distinct node).
"""
import numpy as np

import oracle
import synth
from oracle import forms
from oracle.forms import assemble_vector


def match_by_coords(X_from, X_to, tol=1e-9):
    """perm with X_to[perm] == X_from (rows matched by rounded coordinates)."""
    ka = np.lexsort(np.round(X_from / tol).T[::-1])
    kb = np.lexsort(np.round(X_to / tol).T[::-1])
    perm = np.empty(len(X_from), dtype=np.int64)
    perm[ka] = kb
    err = np.abs(X_from - X_to[perm]).max() if len(X_from) else 0.0
    assert err < 1e-10, f"dof coordinates do not match (max diff {err})"
    return perm


class OracleProblem:
    """Assembled constrained diffusion / mass operators of the oracle on one mesh."""

    def __init__(self, mesh, p, coeff=None, rho=None, q1d=None):
        self.mesh, self.p = mesh, p
        self.q1d = p + 2 if q1d is None else q1d
        self.space = oracle.H1Space(mesh, p)
        self.coords = self.space.dof_coordinates()
        self.K = oracle.assemble(self.space, forms.element_stiffness(mesh, p, self.q1d, coeff))
        self.M = oracle.assemble(self.space, forms.element_mass(mesh, p, self.q1d, rho))
        zero = np.zeros(self.space.ndofs)
        self.Kc, _ = oracle.constrain(self.K, zero, self.space.boundary)
        self.Mc, _ = oracle.constrain(self.M, zero, self.space.boundary)

    def load(self, f):
        b = assemble_vector(self.space, forms.element_load(self.mesh, self.p, self.q1d, f))
        b[self.space.boundary] = 0.0
        return b


def rel_err(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def max_rel_err(a, b):
    """Largest entry error over the largest reference entry: max|a - b| / max|b|."""
    a, b = np.asarray(a), np.asarray(b)
    if a.size == 0:
        return 0.0
    mb = np.abs(b).max()
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0))


def parity_err(a, b):
    """The worse of the norm-wise and the entry-wise relative error, so that one bar
    `parity_err(a, b) <= tol` requires both ||a - b||/||b|| <= tol and
    max|a - b| <= tol * max|b|."""
    return max(rel_err(a, b), max_rel_err(a, b))


def _patch(n, c):
    """Element ids of the 3x3x3 block around element c of an n^3 lattice, and c's position."""
    cx, cy, cz = c % n, (c // n) % n, c // (n * n)
    ids = [ix + n * (iy + n * iz)
           for iz in range(max(cz - 1, 0), min(cz + 2, n))
           for iy in range(max(cy - 1, 0), min(cy + 2, n))
           for ix in range(max(cx - 1, 0), min(cx + 2, n))]
    return ids, ids.index(c)


def on_boundary(X):
    """Nodes on the faces of the unit cube (the essential set)."""
    return np.any((np.abs(X) < 1e-12) | (np.abs(X - 1.0) < 1e-12), axis=1)


def patch_rows(mesh, kappa, p, c, kind, seed):
    """Oracle (A x) of the constrained operator at the dofs of element c of a lattice
    (kappa [E, Q^3] or None for 1),
    from the 3x3x3 element block around c alone, and those dofs' coordinates.

    x = synth.hash_normal(node positions, seed); essential dofs are the nodes on the
    cube's faces: y_b = x_b there, free rows ignore essential columns."""
    n = mesh["n"][0]
    ids, pos = _patch(n, c)
    sub = synth.sub_mesh(mesh, ids)
    space = oracle.H1Space(sub, p)
    coeff = None if kappa is None else kappa[ids]
    if kind == "diffusion":
        Ae = forms.element_stiffness(sub, p, p + 2, coeff)
    else:
        Ae = forms.element_mass(sub, p, p + 2, coeff)
    A = oracle.assemble(space, Ae).tocsr()
    X = space.dof_coordinates()
    ess = on_boundary(X)
    x = synth.hash_normal(X, seed=seed)
    y = A @ np.where(ess, 0.0, x)
    y = np.where(ess, x, y)
    dofs = space.elem_dofs[pos]
    return y[dofs], X[dofs]
