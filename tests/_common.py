"""Helpers shared by the tests: oracle problem setup and dof matching by position.

The library and the oracle number dofs differently; results are compared after
matching dofs by their node coordinates (each H1 dof has a distinct node).
"""
import numpy as np

import oracle
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
